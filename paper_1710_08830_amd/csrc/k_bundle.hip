// Bundle products (hot path): per q,  out = f * V . L . V  (Sec. 3.1 matrix RGE:
// dP = VP Lpp VP with f = 1, dC = 2 VC Lph VC with f = 2), where L is expanded
// from its compact form L[(R1,a,b),(R2,c,d)] = Lc[dR(R1,R2)][(a,b,c,d)].
//
// Small-bundle variant (B <= 64): one workgroup per q, the compact loop and the
// intermediate L.V staged in LDS, and the vertex too when it fits (VLDS);
// arithmetic in T (FP64 or FP32), inputs and outputs in FP64.
#include "common.h"
#include "kernels.h"

namespace tufrg {

template <typename T, bool VLDS>
__global__ __launch_bounds__(256) void bundle_small_kernel(int n_o, int n_ff, int B, int nD,
                                                           const int *__restrict__ didx,
                                                           const double *__restrict__ V,
                                                           const double *__restrict__ Lc, double factor,
                                                           double *__restrict__ out) {
  extern __shared__ unsigned char smem[];
  const int BB = B * B;
  const int no2 = n_o * n_o, no4 = no2 * no2;
  cx<T> *sT = (cx<T> *)smem;
  cx<T> *sL = sT + BB;
  int *sD = (int *)(sL + nD * no4);
  cx<T> *sV = (cx<T> *)(sD + ((n_ff * n_ff + 3) & ~3));
  const int q = blockIdx.x;
  const double *Vq = V + 2 * (size_t)q * BB;
  const double *Lq = Lc + 2 * (size_t)q * nD * no4;
  auto vat = [&](int i) -> cx<T> {
    if constexpr (VLDS) return sV[i];
    return cmake((T)Vq[2 * i], (T)Vq[2 * i + 1]);
  };
  if constexpr (VLDS)
    for (int i = threadIdx.x; i < BB; i += blockDim.x) sV[i] = cmake((T)Vq[2 * i], (T)Vq[2 * i + 1]);
  for (int i = threadIdx.x; i < nD * no4; i += blockDim.x) sL[i] = cmake((T)Lq[2 * i], (T)Lq[2 * i + 1]);
  for (int i = threadIdx.x; i < n_ff * n_ff; i += blockDim.x) sD[i] = didx[i];
  __syncthreads();
  // T = L . V
  for (int idx = threadIdx.x; idx < BB; idx += blockDim.x) {
    const int i = idx / B, j = idx - i * B;
    const int ri = i / no2, ab = i - ri * no2;
    cx<T> s = cmake(T(0), T(0));
    for (int rk = 0; rk < n_ff; ++rk) {
      const cx<T> *Lrow = sL + (size_t)sD[ri * n_ff + rk] * no4 + ab * no2;
      const int vcol = rk * no2 * B + j;
      for (int cd = 0; cd < no2; ++cd) cfma(s, Lrow[cd], vat(vcol + cd * B));
    }
    sT[idx] = s;
  }
  __syncthreads();
  // out = f V . T
  double *oq = out + 2 * (size_t)q * BB;
  for (int idx = threadIdx.x; idx < BB; idx += blockDim.x) {
    const int i = idx / B, j = idx - i * B;
    cx<T> s = cmake(T(0), T(0));
    for (int k = 0; k < B; ++k) cfma(s, vat(i * B + k), sT[k * B + j]);
    oq[2 * idx] = factor * (double)s.re;
    oq[2 * idx + 1] = factor * (double)s.im;
  }
}

hipError_t launch_bundle(int prec, int n_o, int n_ff, int B, int nD, int n_q, const int *didx, const double *V,
                         const double *Lc, double factor, double *out, hipStream_t st) {
  const int no4 = n_o * n_o * n_o * n_o;
  const size_t csz = (prec == 0) ? 16 : 8;
  const size_t base = csz * ((size_t)B * B + (size_t)nD * no4) + sizeof(int) * ((n_ff * n_ff + 3) & ~3);
  const size_t withV = base + csz * (size_t)B * B;
  const size_t limit = 64 * 1024;
  if (base > limit) return hipErrorInvalidValue;
  const bool vlds = withV <= limit;
  const size_t lds = vlds ? withV : base;
  if (prec == 0) {
    if (vlds)
      hipLaunchKernelGGL((bundle_small_kernel<double, true>), dim3(n_q), dim3(256), lds, st, n_o, n_ff, B, nD, didx, V,
                         Lc, factor, out);
    else
      hipLaunchKernelGGL((bundle_small_kernel<double, false>), dim3(n_q), dim3(256), lds, st, n_o, n_ff, B, nD, didx,
                         V, Lc, factor, out);
  } else {
    if (vlds)
      hipLaunchKernelGGL((bundle_small_kernel<float, true>), dim3(n_q), dim3(256), lds, st, n_o, n_ff, B, nD, didx, V,
                         Lc, factor, out);
    else
      hipLaunchKernelGGL((bundle_small_kernel<float, false>), dim3(n_q), dim3(256), lds, st, n_o, n_ff, B, nD, didx,
                         V, Lc, factor, out);
  }
  return hipGetLastError();
}

}  // namespace tufrg

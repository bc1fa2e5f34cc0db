// Bundle products (hot path): per q,  out = f * V . L . V  (Sec. 3.1 matrix RGE:
// dP = VP Lpp VP with f = 1, dC = 2 VC Lph VC with f = 2), where L is expanded
// from its compact form L[(R1,a,b),(R2,c,d)] = Lc[dR(R1,R2)][(a,b,c,d)].
//
// Small-bundle variant (B <= 64): one workgroup per q, the compact loop and the
// intermediate L.V staged in LDS, and the vertex too when it fits (VLDS);
// arithmetic in T (FP64 or FP32), inputs and outputs in FP64.
// Large bundles: two batched complex GEMMs per q (tmp = L.V, out = f V.tmp),
// 64 x 64 output tiles with 16-wide k panels staged in LDS, the loop matrix
// expanded from its compact form while its panel is loaded.
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
  // T = L . V, four adjacent columns per item (B is a multiple of 4: 4 n_ff for
  // two spin-orbitals, the only case with B <= 64)
  const int BQ = B >> 2;
  for (int idx = threadIdx.x; idx < B * BQ; idx += blockDim.x) {
    const int i = idx / BQ, j = (idx - i * BQ) << 2;
    const int ri = i / no2, ab = i - ri * no2;
    cx<T> s0 = cmake(T(0), T(0)), s1 = s0, s2 = s0, s3 = s0;
    for (int rk = 0; rk < n_ff; ++rk) {
      const cx<T> *Lrow = sL + (size_t)sD[ri * n_ff + rk] * no4 + ab * no2;
      const int vcol = rk * no2 * B + j;
      for (int cd = 0; cd < no2; ++cd) {
        const cx<T> l = Lrow[cd];
        const int v = vcol + cd * B;
        cfma(s0, l, vat(v));
        cfma(s1, l, vat(v + 1));
        cfma(s2, l, vat(v + 2));
        cfma(s3, l, vat(v + 3));
      }
    }
    sT[i * B + j] = s0;
    sT[i * B + j + 1] = s1;
    sT[i * B + j + 2] = s2;
    sT[i * B + j + 3] = s3;
  }
  __syncthreads();
  // out = f V . T, four adjacent columns per item
  double *oq = out + 2 * (size_t)q * BB;
  for (int idx = threadIdx.x; idx < B * BQ; idx += blockDim.x) {
    const int i = idx / BQ, j = (idx - i * BQ) << 2;
    cx<T> s0 = cmake(T(0), T(0)), s1 = s0, s2 = s0, s3 = s0;
    for (int k = 0; k < B; ++k) {
      const cx<T> v = vat(i * B + k);
      const cx<T> *Tk = sT + k * B + j;
      cfma(s0, v, Tk[0]);
      cfma(s1, v, Tk[1]);
      cfma(s2, v, Tk[2]);
      cfma(s3, v, Tk[3]);
    }
    const cx<T> r[4] = {s0, s1, s2, s3};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      oq[2 * (i * B + j + c)] = factor * (double)r[c].re;
      oq[2 * (i * B + j + c) + 1] = factor * (double)r[c].im;
    }
  }
}

// C[q] = alpha A[q] Bm[q]; A is the loop expanded from compact form (AL) or dense
template <typename T, bool AL>
__global__ __launch_bounds__(256) void bundle_gemm_kernel(int B, int n_o, int n_ff, int nD,
                                                          const int *__restrict__ didx,
                                                          const double *__restrict__ A,
                                                          const double *__restrict__ Bm, double alpha,
                                                          double *__restrict__ C) {
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ cx<T> sA[TK][TM + 1];
  __shared__ cx<T> sB[TK][TN + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int j0 = blockIdx.x * TN, i0 = blockIdx.y * TM;
  const size_t q = blockIdx.z;
  const int no2 = n_o * n_o, no4 = no2 * no2;
  const size_t BB = (size_t)B * B;
  const double *Aq = AL ? A + 2 * q * (size_t)nD * no4 : A + 2 * q * BB;
  const double *Bq = Bm + 2 * q * BB;
  cx<T> acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = cmake(T(0), T(0));
  for (int k0 = 0; k0 < B; k0 += TK) {
    for (int e = tid; e < TM * TK; e += 256) {
      const int ii = e / TK, kk = e % TK;
      const int i = i0 + ii, k = k0 + kk;
      cx<T> v = cmake(T(0), T(0));
      if (i < B && k < B) {
        size_t src;
        if (AL) {
          const int ri = i / no2, rk = k / no2;
          src = (size_t)didx[ri * n_ff + rk] * no4 + (size_t)(i % no2) * no2 + (k % no2);
        } else {
          src = (size_t)i * B + k;
        }
        v = cmake((T)Aq[2 * src], (T)Aq[2 * src + 1]);
      }
      sA[kk][ii] = v;
    }
    for (int e = tid; e < TK * TN; e += 256) {
      const int kk = e / TN, jj = e % TN;
      const int k = k0 + kk, j = j0 + jj;
      cx<T> v = cmake(T(0), T(0));
      if (k < B && j < B) v = cmake((T)Bq[2 * ((size_t)k * B + j)], (T)Bq[2 * ((size_t)k * B + j) + 1]);
      sB[kk][jj] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TK; ++kk) {
      cx<T> a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = sA[kk][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = sB[kk][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cfma(acc[r][c], a[r], b[c]);
    }
    __syncthreads();
  }
  double *Cq = C + 2 * q * BB;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + ty * 4 + r, j = j0 + tx * 4 + c;
      if (i < B && j < B) {
        Cq[2 * ((size_t)i * B + j)] = alpha * (double)acc[r][c].re;
        Cq[2 * ((size_t)i * B + j) + 1] = alpha * (double)acc[r][c].im;
      }
    }
}

hipError_t launch_bundle(int prec, int n_o, int n_ff, int B, int nD, int n_q, const int *didx, const double *V,
                         const double *Lc, double factor, double *out, double *tmp, hipStream_t st) {
  const int no4 = n_o * n_o * n_o * n_o;
  const size_t csz = (prec == 0) ? 16 : 8;
  const size_t base = csz * ((size_t)B * B + (size_t)nD * no4) + sizeof(int) * ((n_ff * n_ff + 3) & ~3);
  const size_t withV = base + csz * (size_t)B * B;
  const size_t limit = 64 * 1024;
  if (B > 64 || base > limit) {
    if (!tmp) return hipErrorInvalidValue;
    dim3 grid((B + 63) / 64, (B + 63) / 64, n_q), block(256);
    if (prec == 0) {
      hipLaunchKernelGGL((bundle_gemm_kernel<double, true>), grid, block, 0, st, B, n_o, n_ff, nD, didx, Lc, V, 1.0,
                         tmp);
      hipLaunchKernelGGL((bundle_gemm_kernel<double, false>), grid, block, 0, st, B, n_o, n_ff, nD, didx, V, tmp,
                         factor, out);
    } else {
      hipLaunchKernelGGL((bundle_gemm_kernel<float, true>), grid, block, 0, st, B, n_o, n_ff, nD, didx, Lc, V, 1.0,
                         tmp);
      hipLaunchKernelGGL((bundle_gemm_kernel<float, false>), grid, block, 0, st, B, n_o, n_ff, nD, didx, V, tmp,
                         factor, out);
    }
    return hipGetLastError();
  }
  if (B % 4) return hipErrorInvalidValue;  // small bundles are 4 n_ff wide
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

// Integration of the exchange propagators and the per-step reductions.
//
// The single-channel couplings are integrals of the RGE right-hand side over
// the scale (Sec. 3.1); the state is kept in FP64.  Explicit Euler uses
// axpy_max (y = x + h dx together with max |y| and a non-finite flag); the
// Dormand-Prince stages use lincomb and dp_error.  Maxima are taken over
// non-negative doubles, whose bit patterns order like unsigned integers, so
// the atomic max is exact and order-independent.
#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {
constexpr int MAXK = 7;
struct KList {
  const double *k[MAXK];
  double c[MAXK];
};

__device__ inline void block_max_flag(double v, bool bad, unsigned long long *bits, unsigned int *flag) {
  // wave maximum by shuffles, then one value per wave through LDS
  __shared__ double sm[4];
  __shared__ int sb[4];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int anybad = __any(bad);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[wv] = v;
    sb[wv] = anybad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sm[0];
    int b = sb[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      m = fmax(m, sm[i]);
      b |= sb[i];
    }
    atomicMax(bits, (unsigned long long)__double_as_longlong(m));
    if (b) atomicOr(flag, 1u);
  }
}
}  // namespace

__global__ __launch_bounds__(256) void axpy_max_kernel(long long n, const double *__restrict__ x, double h,
                                                       const double *__restrict__ dx, double *__restrict__ y,
                                                       unsigned long long *bits, unsigned int *flag) {
  double m = 0.0;
  bool bad = false;
  const double2 *x2 = (const double2 *)x, *d2 = (const double2 *)dx;
  double2 *y2 = (double2 *)y;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double2 v = x2[i];
    if (dx) {
      const double2 d = d2[i];
      v.x = fma(h, d.x, v.x);
      v.y = fma(h, d.y, v.y);
    }
    if (y) y2[i] = v;
    const double a = sqrt(v.x * v.x + v.y * v.y);
    if (!isfinite(a)) bad = true;
    else m = fmax(m, a);
  }
  block_max_flag(m, bad, bits, flag);
}

hipError_t launch_axpy_max(long long n, const double *x, double h, const double *dx, double *y,
                           unsigned long long *maxbits, unsigned int *flag, hipStream_t st) {
  long long blocks = (n + 255) / 256;
  if (blocks > 512) blocks = 512;  // few blocks: one atomic per block
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(axpy_max_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, x, h, dx, y, maxbits, flag);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void lincomb_kernel(long long n, const double *__restrict__ x, int nk, KList kl,
                                                      double h, double *__restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < nk; ++j) s = fma(kl.c[j], kl.k[j][i], s);
    y[i] = fma(h, s, x[i]);
  }
}

hipError_t launch_lincomb(long long n, const double *x, int nk, const double *const *k, const double *coef,
                          double h, double *y, hipStream_t st) {
  if (nk > MAXK) return hipErrorInvalidValue;
  KList kl;
  for (int j = 0; j < MAXK; ++j) {
    kl.k[j] = j < nk ? k[j] : nullptr;
    kl.c[j] = j < nk ? coef[j] : 0.0;
  }
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(lincomb_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, x, nk, kl, h, y);
  return hipGetLastError();
}

// max over entries (real and imaginary parts separately) of
// |h sum_j e_j k_j| / (atol + rtol max(|x0|, |x1|))
__global__ __launch_bounds__(256) void dp_error_kernel(long long n, const double *__restrict__ x0,
                                                       const double *__restrict__ x1, int nk, KList kl, double h,
                                                       double rtol, double atol, unsigned long long *bits,
                                                       unsigned int *flag) {
  double m = 0.0;
  bool bad = false;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < nk; ++j) s = fma(kl.c[j], kl.k[j][i], s);
    const double sc = atol + rtol * fmax(fabs(x0[i]), fabs(x1[i]));
    const double r = fabs(h * s) / sc;
    if (!isfinite(r)) bad = true;
    else m = fmax(m, r);
  }
  block_max_flag(m, bad, bits, flag);
}

hipError_t launch_dp_error(long long n, const double *x0, const double *x1, int nk, const double *const *k,
                           const double *ecoef, double h, double rtol, double atol, unsigned long long *errbits,
                           unsigned int *flag, hipStream_t st) {
  if (nk > MAXK) return hipErrorInvalidValue;
  KList kl;
  for (int j = 0; j < MAXK; ++j) {
    kl.k[j] = j < nk ? k[j] : nullptr;
    kl.c[j] = j < nk ? ecoef[j] : 0.0;
  }
  long long blocks = (n + 255) / 256;
  if (blocks > 512) blocks = 512;  // few blocks: one atomic per block
  hipLaunchKernelGGL(dp_error_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, x0, x1, nk, kl, h, rtol, atol,
                     errbits, flag);
  return hipGetLastError();
}

__global__ void clear_reduce_kernel(unsigned long long *bits, unsigned int *flag) {
  if (threadIdx.x == 0) {
    *bits = 0ull;
    *flag = 0u;
  }
}

hipError_t launch_clear_reduce(unsigned long long *bits, unsigned int *flag, hipStream_t st) {
  hipLaunchKernelGGL(clear_reduce_kernel, dim3(1), dim3(64), 0, st, bits, flag);
  return hipGetLastError();
}

__global__ void scale_kernel(long long n, const double *__restrict__ x, double s, double *__restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = s * x[i];
}

__global__ void add_kernel(long long n2, const double2 *__restrict__ a, const double2 *__restrict__ b,
                           double2 *__restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x) {
    const double2 u = a[i], v = b[i];
    y[i] = make_double2(u.x + v.x, u.y + v.y);
  }
}

hipError_t launch_add(long long n, const double *a, const double *b, double *y, hipStream_t st) {
  if (n % 2) return hipErrorInvalidValue;  // complex arrays: pairs of doubles
  const long long n2 = n / 2;
  long long blocks = (n2 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n2, (const double2 *)a, (const double2 *)b,
                     (double2 *)y);
  return hipGetLastError();
}

hipError_t launch_scale(long long n, const double *x, double s, double *y, hipStream_t st) {
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, x, s, y);
  return hipGetLastError();
}

}  // namespace tufrg

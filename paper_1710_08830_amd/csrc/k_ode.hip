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
  __shared__ double sm[256];
  __shared__ int sb;
  if (threadIdx.x == 0) sb = 0;
  __syncthreads();
  sm[threadIdx.x] = v;
  if (bad) sb = 1;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(bits, (unsigned long long)__double_as_longlong(sm[0]));
    if (sb) atomicOr(flag, 1u);
  }
}
}  // namespace

__global__ __launch_bounds__(256) void axpy_max_kernel(long long n, const double *__restrict__ x, double h,
                                                       const double *__restrict__ dx, double *__restrict__ y,
                                                       unsigned long long *bits, unsigned int *flag) {
  double m = 0.0;
  bool bad = false;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double r = x[2 * i], im = x[2 * i + 1];
    if (dx) {
      r = fma(h, dx[2 * i], r);
      im = fma(h, dx[2 * i + 1], im);
    }
    if (y) {
      y[2 * i] = r;
      y[2 * i + 1] = im;
    }
    const double a = sqrt(r * r + im * im);
    if (!isfinite(a)) bad = true;
    else m = fmax(m, a);
  }
  block_max_flag(m, bad, bits, flag);
}

hipError_t launch_axpy_max(long long n, const double *x, double h, const double *dx, double *y,
                           unsigned long long *maxbits, unsigned int *flag, hipStream_t st) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
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
  if (blocks > 4096) blocks = 4096;
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

hipError_t launch_scale(long long n, const double *x, double s, double *y, hipStream_t st) {
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, x, s, y);
  return hipGetLastError();
}

}  // namespace tufrg

// Loop surrogate: a multilayer perceptron with GELU activations that maps
// features of (q, Lambda, channel, dR) to one compact loop block, with its
// training (mean-squared loss, reverse-mode gradient, Adam).
//
//   z_l = a_{l-1} W_l^T + b_l,  a_l = GELU(z_l) (not after the last layer),
//   GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2,
//   loss = mean over batch and outputs of (y - t)^2.
//
// All matrix products go through one FP32 tiled GEMM with FP32 accumulation
// (64 x 64 output tile per workgroup, 4 x 4 per thread, k-steps of 16 staged
// in LDS) whose operands may be read transposed, so that the forward product,
// the data gradient dA = dZ W and the weight gradient dW = dZ^T A share it.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace tufrg {

namespace {

constexpr int GT = 64, GK = 16;

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_d(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

}  // namespace

// C[m][n] = sum_k A(m, k) B(k, n) (+ bias[n]) (then GELU, pre-activation to Z)
// A(m, k) = tA ? A[k lda + m] : A[m lda + k];  B(k, n) = tB ? B[n ldb + k] : B[k ldb + n]
__global__ __launch_bounds__(256) void gemm_f32_kernel(int M, int N, int K, const float *__restrict__ A, int lda,
                                                        int tA, const float *__restrict__ B, int ldb, int tB,
                                                        const float *__restrict__ bias, int epi,
                                                        float *__restrict__ C, int ldc, float *__restrict__ Z) {
  __shared__ float sA[GK][GT + 4];
  __shared__ float sB[GK][GT + 4];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int e = tid + 256 * s;
      int m, k;
      if (tA) {
        k = e / GT;
        m = e % GT;
      } else {
        m = e / GK;
        k = e % GK;
      }
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < M && gk < K) v = tA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      sA[k][m] = v;
      int n, kb;
      if (tB) {
        n = e / GK;
        kb = e % GK;
      } else {
        kb = e / GT;
        n = e % GT;
      }
      const int gn = n0 + n, gkb = k0 + kb;
      float w = 0.f;
      if (gn < N && gkb < K) w = tB ? B[(size_t)gn * ldb + gkb] : B[(size_t)gkb * ldb + gn];
      sB[kb][n] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GK; ++k) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tx + 16 * j;
      if (gn >= N) continue;
      float v = acc[i][j];
      if (epi >= 1) v += bias[gn];
      if (epi == 2) {
        Z[(size_t)gm * ldc + gn] = v;
        v = gelu_f(v);
      }
      C[(size_t)gm * ldc + gn] = v;
    }
  }
}

hipError_t launch_gemm_f32(int M, int N, int K, const float *A, int lda, int tA, const float *B, int ldb, int tB,
                           const float *bias, int epi, float *C, int ldc, float *Z, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  hipLaunchKernelGGL(gemm_f32_kernel, grid, dim3(256), 0, st, M, N, K, A, lda, tA, B, ldb, tB, bias, epi, C, ldc,
                     Z);
  return hipGetLastError();
}

// dZ = dA * GELU'(Z), in place on dA
__global__ void gelu_bwd_kernel(long long n, const float *__restrict__ Z, float *__restrict__ dA) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dA[i] *= gelu_d(Z[i]);
}

hipError_t launch_gelu_bwd(long long n, const float *Z, float *dA, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gelu_bwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, Z, dA);
  return hipGetLastError();
}

// db[o] = sum_r dZ[r][o]: partial sums over chunks of CS rows (one thread per
// column and chunk), then a fixed-order sum of the chunks
constexpr int CS = 64;

__global__ void colsum_part_kernel(int rows, int cols, const float *__restrict__ dZ, float *__restrict__ part) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x, ck = blockIdx.y;
  if (o >= cols) return;
  const int r0 = ck * CS, r1 = min(rows, r0 + CS);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += dZ[(size_t)r * cols + o];
  part[(size_t)ck * cols + o] = s;
}

__global__ void colsum_final_kernel(int nck, int cols, const float *__restrict__ part, float *__restrict__ db) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= cols) return;
  float s = 0.f;
  for (int k = 0; k < nck; ++k) s += part[(size_t)k * cols + o];
  db[o] = s;
}

hipError_t launch_colsum(int rows, int cols, const float *dZ, float *part, float *db, hipStream_t st) {
  const int nck = (rows + CS - 1) / CS;
  hipLaunchKernelGGL(colsum_part_kernel, dim3((cols + 63) / 64, nck), dim3(64), 0, st, rows, cols, dZ, part);
  hipLaunchKernelGGL(colsum_final_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, nck, cols, part, db);
  return hipGetLastError();
}

// dY = 2 (Y - T) / (n_elem); loss += sum (Y - T)^2 / n_elem (FP64 atomics)
__global__ void mse_grad_kernel(long long n, const float *__restrict__ Y, const float *__restrict__ T, double inv,
                                float *__restrict__ dY, double *__restrict__ loss) {
  __shared__ double red[256];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (i < n) {
    const float d = Y[i] - T[i];
    dY[i] = (float)(2.0 * inv) * d;
    e2 = (double)d * d;
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] * inv);
}

hipError_t launch_mse_grad(long long n, const float *Y, const float *T, float *dY, double *loss, hipStream_t st) {
  hipLaunchKernelGGL(mse_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, Y, T,
                     1.0 / (double)n, dY, loss);
  return hipGetLastError();
}

// Adam with bias correction: c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ void adam_kernel(long long n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(long long n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, int t, hipStream_t st) {
  const float c1 = (float)(1.0 - pow((double)b1, t)), c2 = (float)(1.0 - pow((double)b2, t));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

// rows of a training batch: dst[r] = src[idx[r]] (row length len)
__global__ void gather_rows_kernel(int rows, int len, const int *__restrict__ idx, const float *__restrict__ src,
                                   float *__restrict__ dst) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)rows * len) return;
  const int r = (int)(i / len), c = (int)(i % len);
  dst[i] = src[(size_t)idx[r] * len + c];
}

hipError_t launch_gather_rows(int rows, int len, const int *idx, const float *src, float *dst, hipStream_t st) {
  const long long n = (long long)rows * len;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows, len, idx, src,
                     dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Loop blocks <-> network rows.  A block is (channel c, coarse q, dR index iD);
// with list pointers null the blocks are all 2 x Nq x nD in compact order
// b = (c Nq + q) nD + iD.

__device__ inline void block_of(long long b, const int *ql, const int *cl, const int *dl, int Nq, int nD, int &q,
                                int &c, int &iD) {
  if (ql) {
    q = ql[b];
    c = cl[b];
    iD = dl[b];
  } else {
    iD = (int)(b % nD);
    q = (int)((b / nD) % Nq);
    c = (int)(b / ((long long)nD * Nq));
  }
}

// features: sin, cos of q and 2q, ln(Lambda) / 5, channel one-hot, dR one-hot
__global__ void sur_features_kernel(long long n, const int *__restrict__ ql, const int *__restrict__ cl,
                                    const int *__restrict__ dl, int Lq, int nD, double lam, float *__restrict__ X) {
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  int q, c, iD;
  block_of(b, ql, cl, dl, Lq * Lq, nD, q, c, iD);
  const int nin = 11 + nD;
  float *x = X + (size_t)b * nin;
  const double tx = 2.0 * M_PI * (double)(q / Lq) / Lq, ty = 2.0 * M_PI * (double)(q % Lq) / Lq;
  x[0] = (float)sin(tx);
  x[1] = (float)cos(tx);
  x[2] = (float)sin(ty);
  x[3] = (float)cos(ty);
  x[4] = (float)sin(2.0 * tx);
  x[5] = (float)cos(2.0 * tx);
  x[6] = (float)sin(2.0 * ty);
  x[7] = (float)cos(2.0 * ty);
  x[8] = (float)(log(lam) / 5.0);
  x[9] = c == 0 ? 1.f : 0.f;
  x[10] = c == 1 ? 1.f : 0.f;
  for (int j = 0; j < nD; ++j) x[11 + j] = j == iD ? 1.f : 0.f;
}

hipError_t launch_sur_features(long long n, const int *ql, const int *cl, const int *dl, int Lq, int nD, double lam,
                               float *X, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sur_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ql, cl, dl, Lq, nD,
                     lam, X);
  return hipGetLastError();
}

// targets: T[b][2 t + r] = s * Lc[c][q][iD][t] (r = real, imaginary), s = Lambda^p / y_scale
__global__ void sur_targets_kernel(long long n, const int *__restrict__ ql, const int *__restrict__ cl,
                                   const int *__restrict__ dl, int Nq, int nD, int no4, double s,
                                   const double *__restrict__ Lc, float *__restrict__ T) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * 2 * no4) return;
  const long long b = i / (2 * no4);
  const int j = (int)(i % (2 * no4));
  int q, c, iD;
  block_of(b, ql, cl, dl, Nq, nD, q, c, iD);
  if (q < 0 || q >= Nq || c < 0 || c > 1 || iD < 0 || iD >= nD) {
    T[i] = __int_as_float(0x7fc00000);  // invalid block: NaN
    return;
  }
  T[i] = (float)(s * Lc[(((size_t)c * Nq + q) * nD + iD) * 2 * no4 + j]);
}

hipError_t launch_sur_targets(long long n, const int *ql, const int *cl, const int *dl, int Nq, int nD, int no4,
                              double s, const double *Lc, float *T, hipStream_t st) {
  const long long tot = n * 2 * no4;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(sur_targets_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, ql, cl, dl, Nq,
                     nD, no4, s, Lc, T);
  return hipGetLastError();
}

// compact loops from network rows of consecutive blocks b0 .. b0 + n - 1 (all-block order):
// Lc[b][t] = (Y[b][2t], Y[b][2t + 1]) * s, s = y_scale / Lambda^p
// Lc = s Y; a non-finite network output sets *bad (if given), so that the
// caller can fall back to the plain loops
__global__ void sur_scatter_kernel(long long n, int no4, double s, const float *__restrict__ Y,
                                   double *__restrict__ Lc, unsigned int *__restrict__ bad) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * 2 * no4) return;
  const float y = Y[i];
  if (bad && !isfinite(y)) atomicOr(bad, 1u);
  Lc[i] = s * (double)y;
}

hipError_t launch_sur_scatter(long long n, int no4, double s, const float *Y, double *Lc, unsigned int *bad,
                              hipStream_t st) {
  const long long tot = n * 2 * no4;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(sur_scatter_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, no4, s, Y, Lc,
                     bad);
  return hipGetLastError();
}

// max |a - b| and max |b| over n complex values (bit patterns of non-negative
// doubles order like the values)
__global__ void sur_compare_kernel(long long n, const double *__restrict__ a, const double *__restrict__ b,
                                   unsigned long long *__restrict__ bits) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0, r = 0.0;
  if (i < n) {
    const double dr = a[2 * i] - b[2 * i], di = a[2 * i + 1] - b[2 * i + 1];
    d = sqrt(dr * dr + di * di);
    r = sqrt(b[2 * i] * b[2 * i] + b[2 * i + 1] * b[2 * i + 1]);
    // a NaN would vanish in the max below: count it as an infinite difference
    if (!(d <= 1.7976931348623157e308)) d = INFINITY;
    if (!(r <= 1.7976931348623157e308)) r = INFINITY;
  }
  // wave-level max, then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) {
    d = fmax(d, __shfl_down(d, off));
    r = fmax(r, __shfl_down(r, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&bits[0], (unsigned long long)__double_as_longlong(d));
    atomicMax(&bits[1], (unsigned long long)__double_as_longlong(r));
  }
}

hipError_t launch_sur_compare(long long n, const double *a, const double *b, unsigned long long *bits,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sur_compare_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, b, bits);
  return hipGetLastError();
}

// max |x| over n floats (bit patterns of non-negative floats order like the values)
__global__ void absmax_f32_kernel(long long n, const float *__restrict__ x, unsigned int *__restrict__ bits) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float v = i < n ? fabsf(x[i]) : 0.f;
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_down(v, off));
  if ((threadIdx.x & 63) == 0) atomicMax(bits, __float_as_uint(v));
}

hipError_t launch_absmax_f32(long long n, const float *x, unsigned int *bits, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(absmax_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, bits);
  return hipGetLastError();
}

}  // namespace tufrg

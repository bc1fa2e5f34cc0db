// Bundle products on the matrix cores for the mixed-precision path (Sec. 3.1
// matrix RGE: dP = VP Lpp VP, dC = 2 VC Lph VC, in the orbital form of
// Sec. 4.2), per coarse q:  tmp = L V,  out = f V tmp.
//
// A complex product is four real ones (Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br)
// and every real operand is split into two BF16 numbers, x = hi + lo with
// hi = RNE(x) and lo = RNE(x - hi); a real product is hi*hi + hi*lo + lo*hi
// on v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the lo*lo term, about
// 2^-18 of the product, is dropped).
//
// Operands live in "split planes": per q four BF16 planes (Re hi, Re lo, Im hi,
// Im lo) of Bp x Bp, Bp = B rounded up to the 96-wide output tile, zero
// outside B x B.  A matrix operand is stored with its rows as plane rows
// (natural); a right operand with its columns as plane rows (transposed), so
// that both matrix-core fragments are 16-byte rows of K.
//   bundle_split_kernel:        V (FP64) -> natural and transposed planes
//   bundle_expand_split_kernel: compact loop (FP64) -> natural planes of L
//   bundle_mfma_kernel<0>:      tmp = L V  -> transposed planes of tmp
//   bundle_mfma_kernel<1>:      out = f V tmp -> FP64
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

constexpr int BT = 96;   // output tile (complex rows x columns) of a workgroup
constexpr int KB = 32;   // K per step
constexpr int LDR = 40;  // LDS row stride in BF16 (80 bytes: conflict-free 16-byte fragment reads)
constexpr int TS = 32;   // transpose tile of the split kernel

// two floats to packed BF16 pairs (round to nearest even): hi and the BF16 of the remainders
__device__ inline void bsplit2(float a, float b, unsigned &hi, unsigned &lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
  const float ra = a - __uint_as_float(hi << 16), rb = b - __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){ra, rb}, bf16x2));
}

__device__ inline bf16x8 negate(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

}  // namespace

size_t bundle_split_pad(int B) { return (size_t)((B + BT - 1) / BT) * BT; }

// V [n_q][B][B] complex FP64 -> natural planes Vn and transposed planes Vt,
// each [n_q][4][Bp][Bp]; one 32 x 32 tile per workgroup
__global__ __launch_bounds__(256) void bundle_split_kernel(int B, int Bp, const double *__restrict__ V,
                                                           unsigned short *__restrict__ Vn,
                                                           unsigned short *__restrict__ Vt) {
  __shared__ unsigned short s[4][TS][TS + 2];
  const int q = blockIdx.z, r0 = blockIdx.y * TS, c0 = blockIdx.x * TS;
  const int t = threadIdx.x, tr = t >> 3, tc = (t & 7) * 4;
  const size_t P = (size_t)Bp * Bp;
  const double *Vq = V + 2 * (size_t)q * B * B;
  float re[4], im[4];
  const int r = r0 + tr;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = c0 + tc + u;
    const bool in = r < B && c < B;
    re[u] = in ? (float)Vq[2 * ((size_t)r * B + c)] : 0.f;
    im[u] = in ? (float)Vq[2 * ((size_t)r * B + c) + 1] : 0.f;
  }
  unsigned rh[2], rl[2], ih[2], il[2];
  bsplit2(re[0], re[1], rh[0], rl[0]);
  bsplit2(re[2], re[3], rh[1], rl[1]);
  bsplit2(im[0], im[1], ih[0], il[0]);
  bsplit2(im[2], im[3], ih[1], il[1]);
  const unsigned pl[4][2] = {{rh[0], rh[1]}, {rl[0], rl[1]}, {ih[0], ih[1]}, {il[0], il[1]}};
  unsigned short *On = Vn + 4 * (size_t)q * P + (size_t)r * Bp + c0 + tc;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    *(u32x2 *)(On + p * P) = (u32x2){pl[p][0], pl[p][1]};
#pragma unroll
    for (int u = 0; u < 4; ++u) s[p][tr][tc + u] = (unsigned short)(pl[p][u >> 1] >> (16 * (u & 1)));
  }
  __syncthreads();
  // transposed: plane row = matrix column c0 + tr, plane columns = matrix rows r0 + tc ..
  unsigned short *Ot = Vt + 4 * (size_t)q * P + (size_t)(c0 + tr) * Bp + r0 + tc;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const unsigned w0 = s[p][tc][tr] | ((unsigned)s[p][tc + 1][tr] << 16);
    const unsigned w1 = s[p][tc + 2][tr] | ((unsigned)s[p][tc + 3][tr] << 16);
    *(u32x2 *)(Ot + p * P) = (u32x2){w0, w1};
  }
}

// compact loop Lc [n_q][nD][n_o^4] complex FP64 -> natural planes Ln [n_q][4][Bp][Bp]
// of L[(R1,a,b)][(R2,c,d)] = Lc[didx(R1,R2)][(a,b,c,d)]; eight columns per thread
__global__ __launch_bounds__(256) void bundle_expand_split_kernel(int n_o, int n_ff, int B, int Bp, int nD, int n_q,
                                                                  const int *__restrict__ didx,
                                                                  const double *__restrict__ Lc,
                                                                  unsigned short *__restrict__ Ln) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int gpr = Bp / 8;
  if (i >= (long long)n_q * Bp * gpr) return;
  const int g = (int)(i % gpr), row = (int)((i / gpr) % Bp), q = (int)(i / ((long long)gpr * Bp));
  const int no2 = n_o * n_o, no4 = no2 * no2;
  const double *Lq = Lc + 2 * (size_t)q * nD * no4;
  float re[8], im[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int col = 8 * g + u;
    re[u] = im[u] = 0.f;
    if (row < B && col < B) {
      const int r1 = row / no2, r2 = col / no2;
      const size_t src = (size_t)didx[r1 * n_ff + r2] * no4 + (size_t)(row - r1 * no2) * no2 + (col - r2 * no2);
      re[u] = (float)Lq[2 * src];
      im[u] = (float)Lq[2 * src + 1];
    }
  }
  u32x4 rh, rl, ih, il;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    unsigned h, l;
    bsplit2(re[2 * u], re[2 * u + 1], h, l);
    rh[u] = h;
    rl[u] = l;
    bsplit2(im[2 * u], im[2 * u + 1], h, l);
    ih[u] = h;
    il[u] = l;
  }
  const size_t P = (size_t)Bp * Bp;
  unsigned short *o = Ln + 4 * (size_t)q * P + (size_t)row * Bp + 8 * g;
  *(u32x4 *)(o) = rh;
  *(u32x4 *)(o + P) = rl;
  *(u32x4 *)(o + 2 * P) = ih;
  *(u32x4 *)(o + 3 * P) = il;
}

// C = A Bm for one q and one 96 x 96 output tile: A in natural planes, Bm in
// transposed planes (both [n_q][4][Bp][Bp]).  OUT 0: C into transposed planes Cs;
// OUT 1: f C into Cd [n_q][B][B] complex FP64.  Four waves in 2 x 2, each a
// 48 x 48 block of 3 x 3 matrix tiles with Re and Im accumulators.
template <int OUT>
__global__ __launch_bounds__(256, 2) void bundle_mfma_kernel(int B, int Bp, int n_q, int tiles,
                                                             const unsigned short *__restrict__ A,
                                                             const unsigned short *__restrict__ Bm, double f,
                                                             unsigned short *__restrict__ Cs,
                                                             double *__restrict__ Cd) {
  // work item: the blocks of one XCD (b % 8) take consecutive items, so the
  // tiles of one q run together on one L2
  const int b = blockIdx.x, per = gridDim.x >> 3;
  const int w = (b & 7) * per + (b >> 3);
  const int tq = tiles * tiles;
  const int q = w / tq;
  if (q >= n_q) return;
  const int t = w - q * tq, i0 = (t / tiles) * BT, j0 = (t - (t / tiles) * tiles) * BT;
  const size_t P = (size_t)Bp * Bp;
  const unsigned short *Aq = A + 4 * (size_t)q * P, *Bq = Bm + 4 * (size_t)q * P;

  __shared__ __align__(16) unsigned short sA[4][BT][LDR];
  __shared__ __align__(16) unsigned short sB[4][BT][LDR];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int fr = lane & 15, fk = 8 * (lane >> 4);

  // staging: per panel 4 planes x 96 rows x 4 granules of 8 K; six per thread
  u32x4 ga[6], gb[6];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int g = tid + 256 * u, p = g / (4 * BT), row = (g >> 2) % BT, kg = g & 3;
      ga[u] = *(const u32x4 *)(Aq + p * P + (size_t)(i0 + row) * Bp + k0 + 8 * kg);
      gb[u] = *(const u32x4 *)(Bq + p * P + (size_t)(j0 + row) * Bp + k0 + 8 * kg);
    }
  };
  auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int g = tid + 256 * u, p = g / (4 * BT), row = (g >> 2) % BT, kg = g & 3;
      *(u32x4 *)&sA[p][row][8 * kg] = ga[u];
      *(u32x4 *)&sB[p][row][8 * kg] = gb[u];
    }
  };

  f32x4 accR[3][3], accI[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n) accR[m][n] = accI[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

  load(0);
  for (int k0 = 0; k0 < Bp; k0 += KB) {
    __syncthreads();  // the previous step's fragments are read
    store();
    __syncthreads();
    if (k0 + KB < Bp) load(k0 + KB);  // in flight during the products
    bf16x8 a[3][4];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int p = 0; p < 4; ++p) a[m][p] = *(const bf16x8 *)&sA[p][wr * 48 + 16 * m + fr][fk];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      bf16x8 bv[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) bv[p] = *(const bf16x8 *)&sB[p][wc * 48 + 16 * n + fr][fk];
      const bf16x8 nih = negate(bv[2]), nil = negate(bv[3]);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        f32x4 r = accR[m][n], im = accI[m][n];
        // Re += Ar Br - Ai Bi
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][0], bv[0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][0], bv[1], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][1], bv[0], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][2], nih, r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][2], nil, r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][3], nih, r, 0, 0, 0);
        // Im += Ar Bi + Ai Br
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][0], bv[2], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][0], bv[3], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][1], bv[2], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][2], bv[0], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][2], bv[1], im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][3], bv[0], im, 0, 0, 0);
        accR[m][n] = r;
        accI[m][n] = im;
      }
    }
  }

  // lane holds rows 4 (lane / 16) + r, column lane % 16 of each matrix tile
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int ib = i0 + wr * 48 + 16 * m + 4 * (lane >> 4), j = j0 + wc * 48 + 16 * n + fr;
      if constexpr (OUT == 0) {
        // transposed planes: row j, the four rows ib.. as four consecutive BF16
        unsigned rh[2], rl[2], ih[2], il[2];
        bsplit2(accR[m][n][0], accR[m][n][1], rh[0], rl[0]);
        bsplit2(accR[m][n][2], accR[m][n][3], rh[1], rl[1]);
        bsplit2(accI[m][n][0], accI[m][n][1], ih[0], il[0]);
        bsplit2(accI[m][n][2], accI[m][n][3], ih[1], il[1]);
        unsigned short *o = Cs + 4 * (size_t)q * P + (size_t)j * Bp + ib;
        *(u32x2 *)(o) = (u32x2){rh[0], rh[1]};
        *(u32x2 *)(o + P) = (u32x2){rl[0], rl[1]};
        *(u32x2 *)(o + 2 * P) = (u32x2){ih[0], ih[1]};
        *(u32x2 *)(o + 3 * P) = (u32x2){il[0], il[1]};
      } else {
        if (j < B) {
          double *o = Cd + 2 * (size_t)q * B * B;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = ib + r;
            if (i < B) {
              o[2 * ((size_t)i * B + j)] = f * (double)accR[m][n][r];
              o[2 * ((size_t)i * B + j) + 1] = f * (double)accI[m][n][r];
            }
          }
        }
      }
    }
}

size_t bundle_split_bytes_per_q(int B) {
  const size_t Bp = bundle_split_pad(B);
  return 4 * 4 * Bp * Bp * sizeof(unsigned short);  // L, V natural, V transposed, tmp transposed
}

// out = f V L V for n_q coarse q, in chunks that fit the workspace ws
// (ws_bytes >= bundle_split_bytes_per_q(B))
hipError_t launch_bundle_bf16x3(int n_o, int n_ff, int B, int nD, int n_q, const int *didx, const double *V,
                                const double *Lc, double factor, double *out, void *ws, size_t ws_bytes,
                                hipStream_t st) {
  const int Bp = (int)bundle_split_pad(B);
  const size_t per_q = bundle_split_bytes_per_q(B);
  if (!ws || ws_bytes < per_q || B < 1) return hipErrorInvalidValue;
  const int chunk = (int)std::min<size_t>((size_t)n_q, ws_bytes / per_q);
  const size_t P4 = 4 * (size_t)Bp * Bp;  // BF16 per q and matrix
  unsigned short *Ln = (unsigned short *)ws, *Vn = Ln + (size_t)chunk * P4, *Vt = Vn + (size_t)chunk * P4,
                 *Ts = Vt + (size_t)chunk * P4;
  const int no4 = n_o * n_o * n_o * n_o;
  const int tiles = Bp / BT;
  for (int q0 = 0; q0 < n_q; q0 += chunk) {
    const int nq = std::min(chunk, n_q - q0);
    const double *Vq = V + 2 * (size_t)q0 * B * B;
    hipLaunchKernelGGL(bundle_split_kernel, dim3(Bp / TS, Bp / TS, nq), dim3(256), 0, st, B, Bp, Vq, Vn, Vt);
    const long long ne = (long long)nq * Bp * (Bp / 8);
    hipLaunchKernelGGL(bundle_expand_split_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, n_o, n_ff, B,
                       Bp, nD, nq, didx, Lc + 2 * (size_t)q0 * nD * no4, Ln);
    const long long items = (long long)nq * tiles * tiles;
    const unsigned nblk = (unsigned)(((items + 7) / 8) * 8);
    hipLaunchKernelGGL(bundle_mfma_kernel<0>, dim3(nblk), dim3(256), 0, st, B, Bp, nq, tiles, Ln, Vt, 1.0, Ts,
                       (double *)nullptr);
    hipLaunchKernelGGL(bundle_mfma_kernel<1>, dim3(nblk), dim3(256), 0, st, B, Bp, nq, tiles, Vn, Ts, factor,
                       (unsigned short *)nullptr, out + 2 * (size_t)q0 * B * B);
  }
  return hipGetLastError();
}

}  // namespace tufrg

// Form-factor projected orbital loops for six spin-orbitals on the matrix
// cores (BF16 split products, FP32 accumulation).
//
// Same quantity as the vector-unit kernel (k_loop_gen.hip):
//   Lc(q)[dR][(a,b,c,d)] = 1/Nf sum_k e^{-ik.dR} sum_m Pi_m(k)_ac W_m(k)_bd,
// with W_m = sum_n L_mn X_n.  Along one kx row the ky sum and the separable ky
// phases form one dense contraction per row:
//   Y[(phi, x)][y] = sum_{ky, m} phi(ky) Pi_m(ky)_x W_m(ky)_y,
// x = (a, c) with a <= c (the other half follows from hermiticity),
// y = (b, d), phi in {1, cos(theta dy), -sin(theta dy)}, theta = 2 pi ky / Lf.
// Written over the reals (K index = (ky, m, re/im)), it is a GEMM of
// (NPHI * 21) x (12 per ky) by (12 per ky) x 72 per row, done with
// v_mfma_f32_16x16x32_bf16 on operands split as v = hi + lo (both BF16) and
// the three products hi*hi + hi*lo + lo*hi accumulated in FP32 (about 16
// significant bits per product).
//
// loop_mfma_kernel: one workgroup (4 waves) per coarse q of one channel; per
//   tile of KT ky it stages Pi, the loop kernels and W in LDS, writes the B
//   operand (W, split) in the lane order of the instruction, and each wave
//   accumulates 3 of the 12 row tiles by 5 column tiles.  At the end of a row
//   the 16 x 16 tiles go to a row buffer Y in HBM.
// loop_rowsum_kernel: per entry pair, Lc[(dx, dy)] = sum_kx e^{-i kx dx} Y(dy)
//   with Y(+-dy) = A +- iB from the cos and -sin rows; writes the same partial
//   layout as the vector-unit kernel.
#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int NO = 6, NO2 = 36, PK = NO * NO2, NC = NO + PK;
constexpr int XC = 21;               // x = (a, c), a <= c
constexpr int NCOL = 72, NT = 5;     // columns (y, re/im); 16-wide column tiles
constexpr int KT = 8;                // ky per tile
constexpr int KS = 12 * KT / 32;     // K steps of 32 per tile
constexpr int NW = 4, NWP = 4, NTHR = 64 * (NW + NWP);  // matrix-core waves, staging waves
constexpr int BFRAG = KS * NT * 64 * 8;  // BF16 values of the B operand of one tile

// x index -> (a, c)
__device__ constexpr int XA[XC] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3, 4, 4, 5};
__device__ constexpr int XCc[XC] = {0, 1, 2, 3, 4, 5, 1, 2, 3, 4, 5, 2, 3, 4, 5, 3, 4, 5, 4, 5, 5};

// packed Hermitian slot of (a, c): diagonal reals first, then Re, Im of lo < hi
__device__ inline void packed_slot(int a, int c, int &re, int &im, float &sgn) {
  if (a == c) {
    re = a;
    im = -1;
    sgn = 0.f;
    return;
  }
  const int lo = a < c ? a : c, hi = a < c ? c : a;
  int p = 0;
  for (int x = 0; x < lo; ++x) p += NO - 1 - x;
  p += hi - lo - 1;
  re = NO + 2 * p;
  im = re + 1;
  sgn = a < c ? 1.f : -1.f;
}

__device__ inline void split(float v, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

// the same for two values, packed as (first | second << 16) for hi and lo
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline void split2(float a, float b, unsigned &hi, unsigned &lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
  const float ra = a - __uint_as_float(hi << 16), rb = b - __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){ra, rb}, bf16x2));
}

// Physical 16-byte granule of the B operand: block blk = (k-step, column tile)
// of 64 granules, granule l = the lane that reads it.  The low four bits of l
// are XOR-ed with a hash of (blk, l / 16): a reading lane group of 16 still
// covers 16 distinct granules, while the stores of the staging waves (scattered
// over columns) spread over more LDS banks.
__device__ inline int bgran(int blk, int l) { return blk * 64 + (l ^ ((7 * blk + 10 * (l >> 4)) & 15)); }

}  // namespace

template <int NDY, int SCHEME>
__global__ __launch_bounds__(NTHR, 1) void loop_mfma_kernel(const float *__restrict__ band,
                                                            const float *__restrict__ kv,
                                                            const float *__restrict__ cvp,
                                                            const float *__restrict__ phy, int Lq, int n_ref,
                                                            int Lf, int q_first, const int *__restrict__ rows,
                                                            int ch, float lam, int deriv, float *__restrict__ Y) {
  constexpr int NPHI = 2 * NDY + 1, ROWS = NPHI * XC, MT = (ROWS + 15) / 16, MTW = (MT + NW - 1) / NW;
  constexpr int SPC = KT * NO * XC * 2;  // floats of one Pi buffer
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index: uniform, keeps the role branches scalar
  const int qrel = blockIdx.x;
  const int qi = rows ? rows[qrel / Lq] * Lq + qrel % Lq : q_first + qrel;
  const int qfx = (qi / Lq) * n_ref, qfy = (qi % Lq) * n_ref;
  const float sg = ch == 0 ? 1.f : -1.f;

  // Two operand buffers (b = tile parity): the Pi values in the A-side layout,
  // the phases and the split B operand.  X and the loop kernels are private to
  // the producer wave that owns their ky and need one buffer.
  __shared__ float sL[KT][NO][NO];         // loop kernels L_mn of each ky
  // X_n(k') packed (transposed for ph), then Pi_m(k)_x for x = (a <= c) of the
  // two buffers, in one array so that a store of either is one address
  __shared__ __align__(16) float sStage[KT * PK + 2 * SPC];
  float(*sX)[PK] = (float(*)[PK])sStage;
  __shared__ float sPh[2][KT][NPHI];       // 1, cos, -sin
  __shared__ __align__(16) __bf16 sBh[2][BFRAG], sBl[2][BFRAG];
  __shared__ int sSlotX[XC][2];            // packed slots (Re, Im) of x = (a <= c); Im < 0 on the diagonal
  __shared__ int sPcOf[NO2];               // packed slot -> float index into the Pi row of (ky, m)
  if (tid < XC) {
    int re, im;
    float sgn;
    packed_slot(XA[tid], XCc[tid], re, im, sgn);
    sSlotX[tid][0] = re;
    sSlotX[tid][1] = im;
    sPcOf[re] = 2 * tid;
    if (im >= 0) sPcOf[im] = 2 * tid + 1;
  }
  // the imaginary parts of the diagonal x stay zero
  for (int i = tid; i < 2 * KT * NO * XC; i += NTHR) sStage[KT * PK + 2 * i + 1] = 0.f;
  // padding columns 72..79 of the last column tile stay zero
  for (int i = tid; i < 2 * KS * 64 * 8; i += NTHR) {
    const int bb = i / (KS * 64 * 8), s = (i / (64 * 8)) % KS, l = (i / 8) % 64, r = i % 8;
    if ((l & 15) >= 8) {
      const int idx = bgran(s * NT + (NT - 1), l) * 8 + r;
      sBh[bb][idx] = (__bf16)0.f;
      sBl[bb][idx] = (__bf16)0.f;
    }
  }
  __syncthreads();

  const int ntk = (Lf + KT - 1) / KT, ntile = Lf * ntk;
  float *Yq = Y + (size_t)qrel * Lf * ROWS * NCOL;

  if (wv >= NW) {
    // ------------------------------------------------------------------
    // Producer wave p: ky rows 2p, 2p + 1 of each tile.  For tile t + 1 it
    // writes Pi and the phases into buffer (t + 1) & 1, evaluates the loop
    // kernels, forms W and writes the B operand; the loads of tile t + 2 are
    // then issued and land while the consumers work on tile t + 1.
    // lane -> one (ky, side) of the wave's rows and packed values p = pl + 16 u
    static_assert(KT == 2 * NWP, "two ky per producer wave");
    const int p = wv - NW;
    constexpr int SPT = (PK + 15) / 16, NDDW = 2 * NO2;  // loop kernel items of one wave
    const int sj = 2 * p + (lane >> 5), sside = (lane >> 4) & 1, pl0 = lane & 15;
    // values of one tile in flight: packed Pi or X, loop kernel inputs (and the
    // shell factors of the momentum-shell scheme), phase
    constexpr bool SHELL = SCHEME == CUT_SHELL;
    struct Pre {
      float v[SPT], e[2][4], c[2][4], ph;
    };
    auto kidx = [&](int kxn, int ky, int side) -> unsigned {
      if (side == 0) return (unsigned)kxn * Lf + ky;
      int kpx = ch == 0 ? qfx - kxn : kxn - qfx;
      kpx += kpx < 0 ? Lf : 0;
      int kpy = ch == 0 ? qfy - ky : ky - qfy;
      kpy += kpy < 0 ? Lf : 0;
      return (unsigned)kpx * Lf + kpy;
    };
    auto fetch = [&](int t, Pre &pr) {
      const int kxn = t / ntk, ky0n = (t - kxn * ntk) * KT;
      {
        const int ky = ky0n + sj < Lf ? ky0n + sj : Lf - 1;
        const float *bp = band + (size_t)kidx(kxn, ky, sside) * NC + NO;
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
          const int pk = pl0 + 16 * u;
          if (pk < PK) pr.v[u] = bp[pk];
        }
      }
      // loop kernel item i = (ky, m, n) of the wave: E_m(k), K_m(k), E_n(k'), K_n(k')
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int i = lane + 64 * v;
        if (i < NDDW) {
          const int j = 2 * p + i / NO2, m = (i / NO) % NO, n = i % NO;
          const int ky = ky0n + j < Lf ? ky0n + j : Lf - 1;
          const unsigned k0 = kidx(kxn, ky, 0), k1 = kidx(kxn, ky, 1);
          pr.e[v][0] = band[(size_t)k0 * NC + m];
          pr.e[v][1] = kv[(size_t)k0 * NO + m];
          pr.e[v][2] = band[(size_t)k1 * NC + n];
          pr.e[v][3] = kv[(size_t)k1 * NO + n];
          if constexpr (SHELL) {
            // (a_m(k), b_m(k), a_n(k'), b_n(k'))
            pr.c[v][0] = cvp[((size_t)k0 * NO + m) * 2];
            pr.c[v][1] = cvp[((size_t)k0 * NO + m) * 2 + 1];
            pr.c[v][2] = cvp[((size_t)k1 * NO + n) * 2];
            pr.c[v][3] = cvp[((size_t)k1 * NO + n) * 2 + 1];
          }
        }
      }
      if (lane < 2 * NPHI) {
        const int j = 2 * p + lane / NPHI, f = lane % NPHI;
        const int kyp = ky0n + j < Lf ? ky0n + j : Lf - 1;
        const float v = f > 0 ? phy[((size_t)kyp * NDY + ((f - 1) % NDY)) * 2 + (f > NDY ? 1 : 0)] : 1.f;
        pr.ph = ky0n + j < Lf ? v : 0.f;  // ky beyond the mesh contributes nothing
      }
    };
    auto stage = [&](int bb, const Pre &pr) {
      // deposit: one LDS store per value, its address chosen per lane (the
      // two sides of the wave go to different arrays)
#pragma unroll
      for (int u = 0; u < SPT; ++u) {
        const int pk = pl0 + 16 * u;
        if (16 * u + 15 < PK || pk < PK) {
          const int m = pk / NO2, pl = pk - NO2 * m;
          const bool flip = sside && ch == 1 && pl >= NO && ((pl - NO) & 1);
          const int po = KT * PK + bb * SPC + 2 * XC * (sj * NO + m) + sPcOf[pl], xo = sj * PK + pk;
          sStage[po + ((xo - po) & -sside)] = flip ? -pr.v[u] : pr.v[u];
        }
      }
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int i = lane + 64 * v;
        if (i < NDDW) {
          float l = sg * divided_difference(pr.e[v][0], -sg * pr.e[v][2], pr.e[v][1], -sg * pr.e[v][3], lam,
                                            dd_scheme(SCHEME), deriv);
          // shell scheme: times a_m(k) b_n(k') + b_m(k) a_n(k')
          if constexpr (SHELL) l *= fmaf(pr.c[v][0], pr.c[v][3], pr.c[v][1] * pr.c[v][2]);
          (&sL[2 * p][0][0])[i] = l;
        }
      }
      if (lane < 2 * NPHI) sPh[bb][2 * p + lane / NPHI][lane % NPHI] = pr.ph;
      // X and the loop kernels of these rows were written by this wave
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // W_m = sum_n L_mn X_n, written straight into the B operand: rows
      // k = (ky, m, re/im), columns (y, re/im), split and in lane order.  For
      // W = wr + i wi the 2 x 2 block of (k re, k im) x (col re, col im) is
      // [[wr, wi], [-wi, wr]].  One item is one chunk of 8 k (4 (ky, m), the
      // 8 values one lane holds for one column; the wave's 12 (ky, m) are
      // chunks 3p .. 3p + 2) and one pair y = (b, d), b <= d: W is Hermitian,
      // so (d, b) takes the conjugate.  Each column is one 16-byte store per
      // operand half.
      static_assert(2 * NO == 3 * 4, "three chunks of 4 (ky, m) per producer wave");
      if (lane < 3 * XC) {
        const int tc = 3 * p + lane / XC, yp = lane % XC;
        const int re = sSlotX[yp][0], im = sSlotX[yp][1], imr = im >= 0 ? im : re;
        // X of this slot for both ky rows of the wave, read once (each read
        // instruction stays within one row)
        float xr[2][NO], xi[2][NO];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int n = 0; n < NO; ++n) {
            xr[jj][n] = sX[2 * p + jj][n * NO2 + re];
            xi[jj][n] = sX[2 * p + jj][n * NO2 + imr];
          }
        unsigned ur[4], ui[4], vr[4], vi[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int jm = 4 * tc + c, j = jm / NO, m = jm % NO;
          const bool j1 = j != 2 * p;
          float wr = 0.f, wi = 0.f;
#pragma unroll
          for (int n = 0; n < NO; ++n) {
            const float l = sL[j][m][n];
            wr = fmaf(l, j1 ? xr[1][n] : xr[0][n], wr);
            wi = fmaf(l, j1 ? xi[1][n] : xi[0][n], wi);
          }
          wi = im >= 0 ? wi : 0.f;
          __bf16 hr, lr, hi, li;
          split(wr, hr, lr);
          split(wi, hi, li);
          ur[c] = __builtin_bit_cast(unsigned short, hr);
          vr[c] = __builtin_bit_cast(unsigned short, lr);
          ui[c] = __builtin_bit_cast(unsigned short, hi);
          vi[c] = __builtin_bit_cast(unsigned short, li);
        }
        const int b = XA[yp], d = XCc[yp], s = tc >> 2, g4 = tc & 3;
        {
          // y = (b, d): column re (wr, -wi), column im (wi, wr)
          const int col = 2 * (b * NO + d), n = col >> 4;
          const int idx = bgran(s * NT + n, g4 * 16 + (col & 15)) * 8;
          const int idx1 = bgran(s * NT + n, g4 * 16 + (col & 15) + 1) * 8;  // column im
          uint4 h0, l0, h1, l1;
          unsigned *ph0 = (unsigned *)&h0, *pl0_ = (unsigned *)&l0, *ph1 = (unsigned *)&h1, *pl1 = (unsigned *)&l1;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            ph0[c] = (ur[c] | (ui[c] << 16)) ^ 0x80000000u;
            pl0_[c] = (vr[c] | (vi[c] << 16)) ^ 0x80000000u;
            ph1[c] = ui[c] | (ur[c] << 16);
            pl1[c] = vi[c] | (vr[c] << 16);
          }
          *(uint4 *)&sBh[bb][idx] = h0;
          *(uint4 *)&sBl[bb][idx] = l0;
          *(uint4 *)&sBh[bb][idx1] = h1;
          *(uint4 *)&sBl[bb][idx1] = l1;
        }
        {
          // y = (d, b) holds the conjugate: column re (wr, wi), column im (-wi, wr).
          // On the diagonal (wi = 0) this rewrites the same two columns with
          // the same values up to the sign of zero.
          const int col = 2 * (d * NO + b), n = col >> 4;
          const int idx = bgran(s * NT + n, g4 * 16 + (col & 15)) * 8;
          const int idx1 = bgran(s * NT + n, g4 * 16 + (col & 15) + 1) * 8;  // column im
          uint4 h0, l0, h1, l1;
          unsigned *ph0 = (unsigned *)&h0, *pl0_ = (unsigned *)&l0, *ph1 = (unsigned *)&h1, *pl1 = (unsigned *)&l1;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            ph0[c] = ur[c] | (ui[c] << 16);
            pl0_[c] = vr[c] | (vi[c] << 16);
            ph1[c] = (ui[c] | (ur[c] << 16)) ^ 0x8000u;
            pl1[c] = (vi[c] | (vr[c] << 16)) ^ 0x8000u;
          }
          *(uint4 *)&sBh[bb][idx] = h0;
          *(uint4 *)&sBl[bb][idx] = l0;
          *(uint4 *)&sBh[bb][idx1] = h1;
          *(uint4 *)&sBl[bb][idx1] = l1;
        }
      }
      // the next stage of this wave rewrites X and the loop kernels
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    // two register sets: the loads of a tile are issued two tiles before it
    // is staged (even tiles in pa, odd tiles in pb)
    Pre pa, pb;
    fetch(0, pa);
    if (1 < ntile) fetch(1, pb);
    stage(0, pa);
    if (2 < ntile) fetch(2, pa);
    __syncthreads();
    for (int t = 0; t < ntile; t += 2) {
      if (t + 1 < ntile) {
        stage(1, pb);
        if (t + 3 < ntile) fetch(t + 3, pb);
      }
      __syncthreads();
      if (t + 1 < ntile) {
        if (t + 2 < ntile) {
          stage(0, pa);
          if (t + 4 < ntile) fetch(t + 4, pa);
        }
        __syncthreads();
      }
    }
  } else {
    // ------------------------------------------------------------------
    // Consumer wave: 3 of the 12 row tiles (phase x Pi rows) by the 5 column
    // tiles, accumulated over a kx row and written to the row buffer at its end
    f32x4 acc[MTW][NT];
    __syncthreads();
    for (int t = 0; t < ntile; ++t) {
      const int bb = t & 1, kx = t / ntk, tk = t - kx * ntk;
      if (tk == 0) {
#pragma unroll
        for (int j = 0; j < MTW; ++j)
#pragma unroll
          for (int n = 0; n < NT; ++n) acc[j][n] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      const float2(*sPc)[XC] = (const float2(*)[XC])(sStage + KT * PK + bb * SPC);
      // A operand (phases times Pi) of this wave's row tiles for k-step s; a
      // row tile past the last (possible for the 3 x 3 box) has a zero A
      // operand and is not written
      auto build_a = [&](int s, bf16x8 (&ah)[MTW], bf16x8 (&al)[MTW]) {
#pragma unroll
        for (int jt = 0; jt < MTW; ++jt) {
          const int mt = wv + NW * jt;
          const int row = mt * 16 + (lane & 15);
          const bool rv = row < ROWS;
          const int f = rv ? row / XC : 0, xi = rv ? row % XC : 0;
          unsigned hp[4], lp[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int jm = 16 * s + 4 * g + r;  // (ky, m) of k = 2 jm (re) and 2 jm + 1 (im)
            const float2 pv = sPc[jm][xi];
            float ph = sPh[bb][jm / NO][f];
            ph = rv ? ph : 0.f;
            split2(ph * pv.x, ph * pv.y, hp[r], lp[r]);
          }
          ah[jt] = __builtin_bit_cast(bf16x8, (u32x4){hp[0], hp[1], hp[2], hp[3]});
          al[jt] = __builtin_bit_cast(bf16x8, (u32x4){lp[0], lp[1], lp[2], lp[3]});
        }
      };
      // per column tile the 3 products hi*hi, hi*lo, lo*hi
      auto products = [&](int s, const bf16x8 (&ah)[MTW], const bf16x8 (&al)[MTW]) {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const int gi = bgran(s * NT + n, lane) * 8;
          const bf16x8 bh = *(const bf16x8 *)&sBh[bb][gi];
          const bf16x8 bl = *(const bf16x8 *)&sBl[bb][gi];
#pragma unroll
          for (int jt = 0; jt < MTW; ++jt)
            acc[jt][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[jt], bh, acc[jt][n], 0, 0, 0);
#pragma unroll
          for (int jt = 0; jt < MTW; ++jt)
            acc[jt][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[jt], bl, acc[jt][n], 0, 0, 0);
#pragma unroll
          for (int jt = 0; jt < MTW; ++jt)
            acc[jt][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[jt], bh, acc[jt][n], 0, 0, 0);
        }
      };
      // software pipeline over the k-steps: the operand of step s + 1 is built
      // while the matrix ops of step s run
      static_assert(KS == 3, "three k-steps per tile");
      bf16x8 ah0[MTW], al0[MTW], ah1[MTW], al1[MTW];
      build_a(0, ah0, al0);
      build_a(1, ah1, al1);
      products(0, ah0, al0);
      build_a(2, ah0, al0);
      products(1, ah1, al1);
      products(2, ah0, al0);
      if (tk == ntk - 1) {
        // row tile (mt, n): lane holds rows 4 g + r, column lane % 16
        float *Yr = Yq + (size_t)kx * ROWS * NCOL;
#pragma unroll
        for (int jt = 0; jt < MTW; ++jt) {
          const int mt = wv + NW * jt;
          if (mt >= MT) break;
#pragma unroll
          for (int n = 0; n < NT; ++n) {
            const int col = n * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = mt * 16 + 4 * g + r;
              if (row < ROWS && col < NCOL) Yr[(size_t)row * NCOL + col] = acc[jt][n][r];
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

// Lc[(dx, dy)] of each entry pair from the rows of Y (see the vector-unit kernel
// for the pair and partial conventions)
template <int NDY>
__global__ __launch_bounds__(256) void loop_rowsum_kernel(const float *__restrict__ Y, const double *__restrict__ tw,
                                                          const int *__restrict__ pairs, int n_pairs, int Lf,
                                                          int nparts, int slot0, int n_slots, int ndx_out,
                                                          float *__restrict__ partial) {
  constexpr int NPHI = 2 * NDY + 1, ROWS = NPHI * XC;
  constexpr int NPT = (NDY == 4) ? 41 : 25;
  const int part = blockIdx.x % nparts, qrel = blockIdx.x / nparts;
  const int pidx = part * blockDim.x + threadIdx.x;
  if (pidx >= n_pairs) return;
  const int tau = pairs[2 * pidx], taub = pairs[2 * pidx + 1];
  constexpr int NO3 = NO * NO2, NO4 = NO2 * NO2;
  const int a = tau / NO3, b = (tau / NO2) % NO, c = (tau / NO) % NO, d = tau % NO;
  int xi = 0;
  for (int x = 0; x < XC; ++x)
    if (XA[x] == a && XCc[x] == c) xi = x;
  const int y = b * NO + d;
  const float *Yq = Y + (size_t)qrel * Lf * ROWS * NCOL;
  float zr[NPT], zi[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) zr[i] = zi[i] = 0.f;
  for (int kx = 0; kx < Lf; ++kx) {
    const float *Yr = Yq + (size_t)kx * ROWS * NCOL + 2 * y;
    float vr[NPHI], vi[NPHI];
#pragma unroll
    for (int f = 0; f < NPHI; ++f) {
      const float2 v = *(const float2 *)(Yr + (size_t)(f * XC + xi) * NCOL);
      vr[f] = v.x;
      vi[f] = v.y;
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      int dx, dy;
      if (NDY == 4) {
        // diamond |dx| + |dy| <= 4, rows dx = -4..4
        int x = -4, s0 = 0;
        while (x < 4 && s0 + 2 * (4 - (x < 0 ? -x : x)) + 1 <= i) {
          s0 += 2 * (4 - (x < 0 ? -x : x)) + 1;
          ++x;
        }
        dx = x;
        dy = i - s0 - (4 - (x < 0 ? -x : x));
      } else {
        dx = i / 5 - 2;
        dy = i % 5 - 2;
      }
      float yr, yi;
      if (dy == 0) {
        yr = vr[0];
        yi = vi[0];
      } else {
        const int ad = dy > 0 ? dy : -dy;
        const float ar = vr[ad], ai = vi[ad], br = vr[NDY + ad], bi = vi[NDY + ad];
        yr = dy > 0 ? ar - bi : ar + bi;
        yi = dy > 0 ? ai + br : ai - br;
      }
      const int adx = dx < 0 ? -dx : dx;
      const int jj = (kx * adx) % Lf;
      const float pr = (float)tw[2 * jj], pi = dx < 0 ? -(float)tw[2 * jj + 1] : (float)tw[2 * jj + 1];
      zr[i] = fmaf(pr, yr, fmaf(-pi, yi, zr[i]));
      zi[i] = fmaf(pr, yi, fmaf(pi, yr, zi[i]));
    }
  }
  const int ndy2 = 2 * NDY + 1;
  const size_t pbase = (size_t)(slot0 + qrel) * (size_t)(ndx_out * ndy2 * NO4);
  (void)n_slots;
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    int dx, dy;
    if (NDY == 4) {
      int x = -4, s0 = 0;
      while (x < 4 && s0 + 2 * (4 - (x < 0 ? -x : x)) + 1 <= i) {
        s0 += 2 * (4 - (x < 0 ? -x : x)) + 1;
        ++x;
      }
      dx = x;
      dy = i - s0 - (4 - (x < 0 ? -x : x));
    } else {
      dx = i / 5 - 2;
      dy = i % 5 - 2;
    }
    if (dx >= 0) {
      const size_t idx = pbase + (size_t)(dx * ndy2 + dy + NDY) * NO4 + tau;
      partial[2 * idx] = zr[i];
      partial[2 * idx + 1] = zi[i];
    }
    if (dx <= 0 && taub != tau) {
      const size_t idx = pbase + (size_t)(-dx * ndy2 - dy + NDY) * NO4 + taub;
      partial[2 * idx] = zr[i];
      partial[2 * idx + 1] = -zi[i];
    }
  }
}

size_t loop_mfma_rowbuf_floats(int ndy, int Lf) {
  const int rows = (2 * ndy + 1) * XC;
  return (size_t)Lf * rows * NCOL;
}

// one channel, coarse q [q_first, q_first + n_q) (or rows): the row buffers Y
// (n_q of them); launch_loop_rowsum then writes the partials to slot (q index
// within the launch) of a one-channel LoopArgs layout
hipError_t launch_loop_mfma(const LoopArgs &a, int ch, float *Y, hipStream_t st) {
  if (a.n_o != 6 || !a.pairs || a.n_pairs <= 0 || !Y) return hipErrorInvalidValue;
  const float *band = (const float *)a.band, *kv = (const float *)a.kv, *phy = (const float *)a.phy;
  const float *cvp = (const float *)a.cv;
  if (a.scheme == CUT_SHELL && !cvp) return hipErrorInvalidValue;
  dim3 grid(a.n_q), block(NTHR);
  const float lam = (float)a.lam;
#define TUFRG_MFMA_LAUNCH(D, S)                                                                                   \
  hipLaunchKernelGGL((loop_mfma_kernel<D, S>), grid, block, 0, st, band, kv, cvp, phy, a.Lq, a.n_ref, a.Lf,     \
                     a.q_first, a.rows, ch, lam, a.deriv, Y)
#define TUFRG_MFMA_SCHEMES(D)                 \
  if (a.scheme == CUT_TEMPERATURE)            \
    TUFRG_MFMA_LAUNCH(D, CUT_TEMPERATURE);    \
  else if (a.scheme == CUT_OMEGA)             \
    TUFRG_MFMA_LAUNCH(D, CUT_OMEGA);          \
  else if (a.scheme == CUT_SHELL)             \
    TUFRG_MFMA_LAUNCH(D, CUT_SHELL);          \
  else                                        \
    return hipErrorInvalidValue;
  if (a.ndx == 5 && a.ndy == 4) {
    TUFRG_MFMA_SCHEMES(4)
  } else if (a.ndx == 3 && a.ndy == 2) {
    TUFRG_MFMA_SCHEMES(2)
  } else {
    return hipErrorInvalidValue;
  }
#undef TUFRG_MFMA_SCHEMES
#undef TUFRG_MFMA_LAUNCH
  return hipGetLastError();
}

hipError_t launch_loop_rowsum(const LoopArgs &a, const float *Y, hipStream_t st) {
  if (a.n_o != 6 || !a.pairs || a.n_pairs <= 0 || !Y) return hipErrorInvalidValue;
  const int np = (a.n_pairs + 255) / 256;
  dim3 g2(a.n_q * np), b2(256);
  if (a.ndy == 4)
    hipLaunchKernelGGL(loop_rowsum_kernel<4>, g2, b2, 0, st, Y, a.tw, a.pairs, a.n_pairs, a.Lf, np, 0, a.n_q, a.ndx,
                       (float *)a.partial);
  else if (a.ndy == 2)
    hipLaunchKernelGGL(loop_rowsum_kernel<2>, g2, b2, 0, st, Y, a.tw, a.pairs, a.n_pairs, a.Lf, np, 0, a.n_q, a.ndx,
                       (float *)a.partial);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace tufrg

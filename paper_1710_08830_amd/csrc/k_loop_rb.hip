// Form-factor projected orbital loops for six spin-orbitals on the matrix
// cores (BF16 split products, FP32 accumulation), written in a real basis of
// Hermitian matrices.
//
// The loop entry (Sec. 3.1 loop matrices in the orbital form of Sec. 4.2)
//   Lc(q)[dR][(a,b,c,d)] = 1/Nf sum_k e^{-ik.dR} sum_m Pi_m(k)_ac W_m(k)_bd,
//   W_m = sum_n L_mn X_n,  X_n = Pi_n(k') (pp, k' = q - k) or Pi_n(k')^T (ph, k' = k - q),
// pairs two Hermitian 6 x 6 matrices.  In the real basis E^alpha of Hermitian
// matrices (alpha < 6: e_a e_a^T; then for each pair a < c: e_a e_c^T + e_c e_a^T
// and i (e_a e_c^T - e_c e_a^T)), whose coordinates are the packed projector
// values of the band data, Pi_m = sum_alpha pi_m^alpha E^alpha and
// W_m = sum_beta w_m^beta E^beta with real coordinates, so
//   sum_m Pi_m(k)_ac W_m(k)_bd = sum_{alpha,beta} mu^{alpha beta}(k) E^alpha_ac E^beta_bd,
//   mu^{alpha beta}(k) = sum_m pi_m^alpha(k) w_m^beta(k)      (36 x 36, real).
// The k sum then acts on a real 36 x 36 matrix per k instead of 1296 complex
// entries, and lambda(-dR) = conj lambda(dR) (mu is real), so only the half
// plane dx > 0 or (dx = 0, dy >= 0) is summed.
//
// Separable phases.  Along a kx row the ky sum with the phases
// phi in {1, cos(theta dy), sin(theta dy)}, dy = 1..NDY, theta = 2 pi ky / Lf,
// is one dense contraction, and the A operand (phases times pi) does not
// depend on q:
//   Y[(phi, alpha)][(q, beta)] = sum_{ky, m} phi(ky) pi_m^alpha(ky) w_m^beta(ky; q).
// loop_rb_apre_kernel: the A operand (phase rows times pi, split), which
//   depends on neither q, Lambda nor the channel, once per context in the
//   lane order of the matrix instruction.
// loop_rb_kernel: one workgroup (eight waves, two per SIMD) per group of four
//   coarse q of one channel and a block of kx rows.  Per tile of 16 ky
//   (K = 96 = (ky, m)) it evaluates the loop kernels L_mn and forms the B
//   operand w (split) in LDS for the next tile, while each wave loads the A
//   fragments of its row tiles (L2-resident) and runs the three BF16 products
//   (hi*hi + hi*lo + lo*hi, v_mfma_f32_16x16x32_bf16) into 16 x 16 FP32 tiles
//   (rows: 9 x 36 phase rows; columns: 4 q x 36 beta).  At the end of a kx
//   row the tiles go to a row buffer Y.
//   Kramers pairs (PAIR): when bands (0,1), (2,3), (4,5) are degenerate at
//   every k, L_mn depends on the pairs only and the band sum groups into three
//   pairs with summed projectors; a tile then covers 16 ky pairs, the six K
//   values of a pair point being (ky - 2 v) 3 + pair, with the same B layout
//   and matrix ops over half as many tiles.
// loop_rb_rowsum_kernel: the kx sum with the kx phases, in FP64, for the half
//   plane of difference vectors: lambda^{alpha beta}(q, dR).
// loop_rb_finalize_kernel: back from the real basis to the entries (a,b,c,d),
//   the other half plane by conjugation, times 1/Nf: the compact loops.
#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int NO = 6;               // spin-orbitals
constexpr int NA = 36;              // real coordinates of a Hermitian 6 x 6 matrix
constexpr int PK = NO * NA;         // packed projector values of all bands at one k
constexpr int NC = NO + PK;         // band values per k: e_m, then pi_m^alpha
constexpr int NQG = 4;              // coarse q per workgroup
constexpr int NCOL = NQG * NA;      // columns (q, beta)
constexpr int NCT = NCOL / 16;      // column tiles
constexpr int KT = 16;              // ky per tile
constexpr int KTOT = KT * NO;       // K = (ky, m) per tile
constexpr int KS = KTOT / 32;       // K steps of 32
constexpr int NW = 8, NTHR = 64 * NW;
constexpr int PIS = KTOT + 4;       // LDS row stride of pi (floats): 16-byte rows, spread banks
constexpr int NBT = 8;              // B-building threads per (q, ky): beta sets of 5, 5, 5, 5, 4, 4, 4, 4
constexpr int NBS = 5;
constexpr int NDD = (NQG * KT * NO * NO + NTHR - 1) / NTHR;  // loop kernels per thread and tile
constexpr int NPIF = (KT * PK + NTHR - 1) / NTHR;             // pi values staged per thread and tile
constexpr int NEV = KT * (1 + NQG) * 2 * NO;                  // e, K at k and at the four k'
static_assert(NCOL % 16 == 0 && KTOT % 32 == 0, "tile shape");
static_assert(NTHR == NQG * KT * NBT, "one B-building thread per (q, ky, beta set)");

template <int NDY>
struct RB {
  static constexpr int NPHI = 2 * NDY + 1;          // 1, cos dy, sin dy
  static constexpr int ROWS = NPHI * NA;            // (phi, alpha), phi-major
  static constexpr int MT = (ROWS + 15) / 16;       // row tiles
  static constexpr int MTW = (MT + NW - 1) / NW;    // row tiles per wave (wave w: w, w + 8, ...)
};

// two floats to packed BF16 (round to nearest even) and the BF16 of the remainders
__device__ inline void split2(float a, float b, unsigned &hi, unsigned &lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
  const float ra = a - __uint_as_float(hi << 16), rb = b - __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){ra, rb}, bf16x2));
}

// byte offset of the BF16 pair (K, K + 1), K even, of column col in the B
// operand of one buffer: granules of 8 K (16 bytes) in the lane order of the
// matrix instruction (lane = 16 (K % 32) / 8 + col % 16), blocks of 64
// granules per (K step, column tile)
__device__ inline int bpair_off(int K, int col) {
  const int s = K >> 5, kk = K & 31;
  const int gr = ((s * NCT + (col >> 4)) << 6) + ((kk >> 3) << 4) + (col & 15);
  return (gr << 4) + ((kk & 7) << 1);
}

}  // namespace

// The A operand Y's left factor, phi(ky) pi_m^alpha(k) split, does not depend
// on q, Lambda or the channel: computed once per context, in the lane order of
// the matrix instruction, as [kx][ky tile][K step][row tile][hi, lo][lane] of
// 8 BF16 (16 bytes): lane l holds row 16 mt + l % 16 and K = 32 s + 8 (l / 16)
// .. + 7 of the tile, K = (ky - 16 tile) 6 + m (paired: K = (v - 16 tile) 6 +
// 3 (ky - 2 v) + pair, with the pair sums of the projectors); rows past the
// 9 x 36 and ky past the mesh are zero.  The split is that of the FP32 product (the
// compiler may form the remainder from the unrounded product, a last-bit
// difference of lo: loops agree with an in-kernel build to about 2e-9).
template <int NDY, bool PAIR>
__global__ __launch_bounds__(256) void loop_rb_apre_kernel(const float *__restrict__ band,
                                                           const float *__restrict__ pir,
                                                           const float *__restrict__ phy, int Lf,
                                                           u32x4 *__restrict__ apre) {
  using S = RB<NDY>;
  const int ntk = ((PAIR ? Lf / 2 : Lf) + KT - 1) / KT;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)Lf * ntk * KS * S::MT * 64;
  if (gid >= total) return;
  const int lane = (int)(gid % 64);
  long long r = gid / 64;
  const int mt = (int)(r % S::MT);
  r /= S::MT;
  const int s = (int)(r % KS);
  r /= KS;
  const int tk = (int)(r % ntk), kx = (int)(r / ntk);
  const int row = mt * 16 + (lane & 15), ph = row / NA, alpha = row % NA;
  float v[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    // K = (v, m'): point v of the tile, band m' (paired: ky = 2 v + m' / 3 and
    // the pair m' % 3)
    const int K = 32 * s + 8 * (lane >> 4) + t, vk = tk * KT + K / NO, mv = K % NO;
    const int ky = PAIR ? 2 * vk + mv / 3 : vk, m = PAIR ? mv % 3 : mv;
    float f = 0.f, pv = 0.f;
    if (row < S::ROWS && ky < Lf) {
      f = ph == 0 ? 1.f : ph <= NDY ? phy[((size_t)ky * NDY + ph - 1) * 2] : -phy[((size_t)ky * NDY + ph - NDY - 1) * 2 + 1];
      pv = PAIR ? pir[((size_t)kx * Lf + ky) * (3 * NA) + m * NA + alpha]
                : band[((size_t)kx * Lf + ky) * NC + NO + m * NA + alpha];
    }
    v[t] = pv * f;
  }
  u32x4 h, l;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    unsigned hh, ll;
    split2(v[2 * t], v[2 * t + 1], hh, ll);
    h[t] = hh;
    l[t] = ll;
  }
  const size_t o = ((((size_t)kx * ntk + tk) * KS + s) * S::MT + mt) * 2 * 64 + lane;
  apre[o] = h;
  apre[o + 64] = l;
}

template <int NDY, int SCHEME, bool PAIR>
__global__ __launch_bounds__(NTHR, 1) void loop_rb_kernel(
    const float *__restrict__ band, const float *__restrict__ pir, const float *__restrict__ kv,
    const float *__restrict__ cvp, const bf16x8 *__restrict__ apre, int Lq, int n_ref, int Lf, int q_first,
    int n_q, const int *__restrict__ rows, int ch, float lam, int deriv, int n_groups, int n_kxb, int kxr,
    float *__restrict__ Y) {
  using S = RB<NDY>;
  constexpr int MT = S::MT, MTW = S::MTW, ROWS = S::ROWS;
  constexpr bool SHELL = SCHEME == CUT_SHELL;
  constexpr int PER = SHELL ? 4 * NO : 2 * NO;  // band values per point: e, K (shell: and a, b)
  constexpr int NEVU = ((1 + NQG) * PER + 63) / 64;  // per-lane values of one ky row of sE

  // work item: XCD x takes the kx blocks x, x + 8, ..., the groups of q
  // fastest, so that the workgroups running at once on one XCD share the kx
  // rows of the A operand in its L2
  const int b = blockIdx.x, xcd = b & 7, j = b >> 3;
  const int g = j % n_groups, kxb = xcd + 8 * (j / n_groups);
  if (kxb >= n_kxb) return;
  const int kx0 = kxb * kxr, nrow = min(kxr, Lf - kx0);
  // points v of a kx row: each ky (six bands), or paired: ky 2 v and 2 v + 1
  // with three pairs each, as six bands m' = 3 (ky - 2 v) + pair
  const int ntk = ((PAIR ? Lf / 2 : Lf) + KT - 1) / KT, ntile = nrow * ntk;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  // the two waves that share a SIMD take opposite orders of their matrix
  // products and B-operand work, so one's vector work runs beside the other's
  // matrix ops
  const bool mfma_first = ((wv & 1) ^ (wv >> 2)) == 0;

  __shared__ __align__(16) unsigned char sB[2][2][KS * NCT * 64 * 16];  // [buffer][hi, lo] granules
  __shared__ __align__(16) float sL[NQG][KT][NO * NO];                    // loop kernels L_mn
  // e_m, K_m at (kx, ky) [slot 0] and at k'(q, ky) [slots 1..4]; shell: then
  // (a_m, b_m); two tiles (staged one tile ahead of their loop kernels)
  __shared__ __align__(16) float sE[2][KT][1 + NQG][PER];
  __shared__ int sQf[1 + NQG][2];  // fine-mesh offsets of the group's q (slot 0: zero)

  if (tid <= NQG) {
    int qfx = 0, qfy = 0;
    if (tid > 0) {
      const int qidx = NQG * g + tid - 1;
      const int qc = qidx < n_q ? qidx : n_q - 1;  // past the list: any valid q (zero column)
      const int q = rows ? rows[qc / Lq] * Lq + qc % Lq : q_first + qc;
      qfx = (q / Lq) * n_ref;
      qfy = (q % Lq) * n_ref;
    }
    sQf[tid][0] = qfx;
    sQf[tid][1] = qfy;
  }
  __syncthreads();
  // k' of slot s (1..4) at (kx, ky); slot 0: k itself
  auto kpt = [&](int qfx, int qfy, bool self, int kx, int ky) __attribute__((always_inline)) {
    if (self) return kx * Lf + ky;
    int kpx = ch == 0 ? qfx - kx : kx - qfx;
    kpx += kpx < 0 ? Lf : 0;
    int kpy = ch == 0 ? qfy - ky : ky - qfy;
    kpy += kpy < 0 ? Lf : 0;
    return kpx * Lf + kpy;
  };

  // ---- per-thread constants -------------------------------------------------
  // band values: lane index i = lane + 64 u < (1 + NQG) PER: slot, kind, band
  int ev_slot[NEVU], ev_off[NEVU], ev_dky[NEVU];
  const float *ev_src[NEVU];
  int ev_stride[NEVU];
#pragma unroll
  for (int u = 0; u < NEVU; ++u) {
    const int i = min(lane + 64 * u, (1 + NQG) * PER - 1);
    // per slot: e_0..e_5, K_0..K_5, then (shell) a_0, b_0, a_1, b_1, ... as in cvp
    const int slot = i / PER, r = i % PER, kind = r < NO ? 0 : r < 2 * NO ? 1 : 2;
    const int off = r - NO * kind, mv = kind == 2 ? off / 2 : off;
    // paired: band m' is the first band 2 (m' % 3) of a pair at ky 2 v + m' / 3
    const int mb = PAIR ? 2 * (mv % 3) : mv;
    ev_slot[u] = slot;
    ev_off[u] = kind == 2 ? 2 * mb + (off & 1) : mb;
    ev_dky[u] = PAIR ? mv / 3 : 0;
    ev_src[u] = kind == 0 ? band : kind == 1 ? kv : cvp;
    ev_stride[u] = kind == 0 ? NC : kind == 1 ? NO : 2 * NO;
  }
  // loop kernels and B operand: thread (q column dq, ky dky, part dsub)
  const int dq = tid / (KT * NBT), dky = (tid / NBT) % KT, dsub = tid % NBT;
  const int nb = dsub < 4 ? 5 : 4, be0 = dsub < 4 ? 5 * dsub : 20 + 4 * (dsub - 4);
  const int bqfx = sQf[1 + dq][0], bqfy = sQf[1 + dq][1];
  // B-operand byte offsets: column part per beta, K part per band pair
  int bcol[NBS], bk[NO / 2];
#pragma unroll
  for (int i = 0; i < NBS; ++i) {
    const int col = dq * NA + be0 + min(i, nb - 1);
    bcol[i] = ((col >> 4) << 10) + ((col & 15) << 4);
  }
#pragma unroll
  for (int mp = 0; mp < NO / 2; ++mp) {
    const int K = dky * NO + 2 * mp, kk = K & 31;
    bk[mp] = (((K >> 5) * NCT) << 10) + ((kk >> 3) << 8) + ((kk & 7) << 1);
  }
  const float sg = ch == 0 ? 1.f : -1.f;

  // band values of the wave's two ky of a tile (for the loop kernels)
  struct Pre {
    float ev[2][NEVU];
  };
  auto fetch = [&](int t, Pre &pr) __attribute__((always_inline)) {
    const int kx = kx0 + t / ntk, ky0 = (t - (t / ntk) * ntk) * KT;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int v = ky0 + 2 * wv + kk;
#pragma unroll
      for (int u = 0; u < NEVU; ++u) {
        const int sl = ev_slot[u];
        // ky past the mesh: any point (zero A rows)
        const int ky = min(PAIR ? 2 * v + ev_dky[u] : v, Lf - 1);
        const int k = kpt(sQf[sl][0], sQf[sl][1], sl == 0, kx, ky);
        pr.ev[kk][u] = ev_src[u][(size_t)k * ev_stride[u] + ev_off[u]];
      }
    }
  };
  auto stage = [&](const Pre &pr, int eb) __attribute__((always_inline)) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int u = 0; u < NEVU; ++u)
        if (lane + 64 * u < (1 + NQG) * PER) (&sE[eb][2 * wv + kk][0][0])[lane + 64 * u] = pr.ev[kk][u];
  };
  // loop kernels L_mn of this thread's (q, ky): (m, n) = divmod(dsub + 8 i, 6).
  // The eight threads of one (q, ky) are lanes of one wave, and so are those
  // that read these L_mn for the B operand: no barrier between the two.
  auto loop_kernels = [&](int eb) __attribute__((always_inline)) {
    const float *e0 = sE[eb][dky][0], *e1 = sE[eb][dky][1 + dq];
    // paired: only the two diagonal 3 x 3 blocks (bands of the same ky)
    constexpr int NMN = PAIR ? 18 : NO * NO;
#pragma unroll
    for (int i = 0; i < (NMN + NBT - 1) / NBT; ++i) {
      const int j = dsub + NBT * i;
      if (j < NMN) {
        const int m = PAIR ? 3 * (j / 9) + (j % 9) / 3 : j / NO;
        const int n = PAIR ? 3 * (j / 9) + j % 3 : j - NO * (j / NO);
        const int mn = NO * m + n;
        float l = sg * divided_difference(e0[m], -sg * e1[n], e0[NO + m], -sg * e1[NO + n], lam, dd_scheme(SCHEME),
                                          deriv);
        if constexpr (SHELL) l *= fmaf(e0[2 * NO + 2 * m], e1[2 * NO + 2 * n + 1], e0[2 * NO + 2 * m + 1] * e1[2 * NO + 2 * n]);
        sL[dq][dky][mn] = l;
      }
    }
  };
  // B operand: w_m^beta = sum_n L_mn X_n^beta for this thread's (q, ky) and
  // beta set, split, as BF16 pairs (m, m + 1) of the columns (q, beta); a q
  // past the end of the list repeats the last one (its columns are never
  // read).  ph takes the transpose of X, whose imaginary coordinates change
  // sign: applied to the columns in the kx sums (the products are linear and
  // the rounding symmetric, so the result is the same).
  auto build_b = [&](int bb, int t) __attribute__((always_inline)) {
    // packed X_n(k') of this thread's (q, ky) and beta set (L2-resident rows;
    // the load latency is covered by the matrix ops of the other wave of
    // the SIMD)
    float xi[NO][NBS];
    {
      const int kx = kx0 + t / ntk, v = (t - (t / ntk) * ntk) * KT + dky;
      if constexpr (PAIR) {
        // pair sums of the projectors at k' of ky 2 v and 2 v + 1
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int ky = min(2 * v + h, Lf - 1);
          const float *src = pir + (size_t)kpt(bqfx, bqfy, false, kx, ky) * (3 * NA) + be0;
#pragma unroll
          for (int n = 0; n < 3; ++n)
#pragma unroll
            for (int i = 0; i < NBS; ++i) xi[3 * h + n][i] = src[n * NA + min(i, nb - 1)];
        }
      } else {
        const int ky = min(v, Lf - 1);
        const float *src = band + (size_t)kpt(bqfx, bqfy, false, kx, ky) * NC + NO + be0;
#pragma unroll
        for (int n = 0; n < NO; ++n)
#pragma unroll
          for (int i = 0; i < NBS; ++i) xi[n][i] = src[n * NA + min(i, nb - 1)];
      }
    }
    unsigned char *bh = sB[bb][0], *bl = sB[bb][1];
#pragma unroll
    for (int mp = 0; mp < NO / 2; ++mp) {
      const f32x2 *Lr0 = (const f32x2 *)&sL[dq][dky][2 * mp * NO];
      const f32x2 *Lr1 = (const f32x2 *)&sL[dq][dky][(2 * mp + 1) * NO];
      float L0[NO], L1[NO];
#pragma unroll
      for (int n = 0; n < NO; n += 2) {
        const f32x2 a0 = Lr0[n / 2], a1 = Lr1[n / 2];
        L0[n] = a0[0];
        L0[n + 1] = a0[1];
        L1[n] = a1[0];
        L1[n + 1] = a1[1];
      }
#pragma unroll
      for (int i = 0; i < NBS; ++i) {
        // the fifth beta of the 4-sets repeats the fourth: same value, same address
        float w0 = 0.f, w1 = 0.f;
#pragma unroll
        for (int n = 0; n < NO; ++n) {
          // paired: L_{m'n'} vanishes between bands of different ky
          if (!PAIR || n / 3 == (2 * mp) / 3) w0 = fmaf(L0[n], xi[n][i], w0);
          if (!PAIR || n / 3 == (2 * mp + 1) / 3) w1 = fmaf(L1[n], xi[n][i], w1);
        }
        unsigned h, l;
        split2(w0, w1, h, l);
        const int off = bcol[i] + bk[mp];
        *(unsigned *)(bh + off) = h;
        *(unsigned *)(bl + off) = l;
      }
    }
  };

  f32x4 acc[MTW][NCT];
  // A fragments of the first K step of the tile about to be multiplied: the
  // last K step of each tile loads those of the next, so they arrive during
  // that step's products, the B-operand work and the barriers
  bf16x8 ah[MTW], al[MTW];
  auto load_a = [&](int t, int s, bf16x8 *h, bf16x8 *l) __attribute__((always_inline)) {
    // tiles are stored in work order: tile t of this item at kx0 * ntk + t
    const bf16x8 *ab = apre + (((size_t)kx0 * ntk + t) * KS + s) * MT * 128 + lane;
#pragma unroll
    for (int jt = 0; jt < MTW; ++jt)
      if (wv + NW * jt < MT) {
        const int mt = wv + NW * jt;
        h[jt] = ab[(size_t)mt * 128];
        l[jt] = ab[(size_t)mt * 128 + 64];
      }
  };

  // products of tile t (B operand in buffer bb) for this wave's row tiles; the
  // A fragments of each K step come from the precomputed operand (in L2), the
  // next step's loads (at the last step: the next tile's first) in flight
  // during the current step's products
  auto mfma_tile = [&](int bb, int t) __attribute__((always_inline)) {
    const unsigned char *bh = sB[bb][0], *bl = sB[bb][1];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bf16x8 nh[MTW], nl[MTW];
      if (s + 1 < KS)
        load_a(t, s + 1, nh, nl);
      else if (t + 1 < ntile)
        load_a(t + 1, 0, nh, nl);
      // column tiles in order, the B fragments of the next one loaded while
      // the products of this one run (no further hoisting: the scheduling
      // barrier keeps the live B fragments at two)
      const int gb = ((s * NCT) << 10) + (lane << 4);
      bf16x8 bhv = *(const bf16x8 *)(bh + gb), blv = *(const bf16x8 *)(bl + gb);
#pragma unroll
      for (int n = 0; n < NCT; ++n) {
        bf16x8 bhn = bhv, bln = blv;
        if (n + 1 < NCT) {
          bhn = *(const bf16x8 *)(bh + gb + ((n + 1) << 10));
          bln = *(const bf16x8 *)(bl + gb + ((n + 1) << 10));
        }
#pragma unroll
        for (int jt = 0; jt < MTW; ++jt) {
          if (wv + NW * jt < MT) {
            acc[jt][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[jt], bhv, acc[jt][n], 0, 0, 0);
            acc[jt][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[jt], blv, acc[jt][n], 0, 0, 0);
            acc[jt][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[jt], bhv, acc[jt][n], 0, 0, 0);
          }
        }
        bhv = bhn;
        blv = bln;
        __builtin_amdgcn_sched_barrier(0);
      }
      if (s + 1 < KS || t + 1 < ntile) {
#pragma unroll
        for (int jt = 0; jt < MTW; ++jt) {
          ah[jt] = nh[jt];
          al[jt] = nl[jt];
        }
      }
    }
  };
  // end of kx row: tile (mt, n), lane holds rows 4 lg + r, column lane % 16
  const int lg = lane >> 4;
  auto write_row = [&](int kx) __attribute__((always_inline)) {
    float *Yr = Y + ((size_t)g * Lf + kx) * ROWS * NCOL;
#pragma unroll
    for (int jt = 0; jt < MTW; ++jt) {
      const int mt = wv + NW * jt;
      if (mt < MT) {
#pragma unroll
        for (int n = 0; n < NCT; ++n) {
          const int col = n * 16 + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = mt * 16 + 4 * lg + r;
            if (row < ROWS) Yr[(size_t)row * NCOL + col] = acc[jt][n][r];
          }
        }
      }
    }
  };

  // prologue: tile 0 staged and its B operand built, tile 1 in flight
  Pre pr;
  // prologue: tiles 0 and 1 staged, the B operand of tile 0 built, tile 2 in
  // flight
  load_a(0, 0, ah, al);
  fetch(0, pr);
  stage(pr, 0);
  if (1 < ntile) {
    fetch(1, pr);
    stage(pr, 1);
  }
  __syncthreads();
  loop_kernels(0);
  build_b(0, 0);
  if (2 < ntile) fetch(2, pr);
  __syncthreads();
  int t = 0;
  for (int r = 0; r < nrow; ++r) {
#pragma unroll
    for (int jt = 0; jt < MTW; ++jt)
#pragma unroll
      for (int n = 0; n < NCT; ++n) acc[jt][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int tk = 0; tk < ntk; ++tk, ++t) {
      // LDS holds B of tile t (buffer bb) and the band values of tile t + 1
      // (buffer (t + 1) & 1); registers those of tile t + 2.  One barrier per
      // tile: the vector work for tile t + 1 (loop kernels, B operand, staging
      // of tile t + 2) of one wave of a SIMD runs beside the other's matrix ops
      const int bb = t & 1;
      auto vector_work = [&]() __attribute__((always_inline)) {
        if (t + 1 < ntile) {
          loop_kernels(bb ^ 1);
          build_b(bb ^ 1, t + 1);
        }
        if (t + 2 < ntile) stage(pr, bb);
        // band values of tile t + 3: in flight during the matrix ops and the
        // barrier
        if (t + 3 < ntile) fetch(t + 3, pr);
      };
      if (!mfma_first) vector_work();
      mfma_tile(bb, t);
      if (mfma_first) vector_work();
      __syncthreads();
    }
    write_row(kx0 + r);
  }
}

// ---------------------------------------------------------------------------
// kx sums: lambda^{alpha beta}(q, dR) for the half plane of the computed
// shape, FP64.  With A_dy = sum_ky cos(ky dy theta) mu and S_dy = sum_ky
// sin(ky dy theta) mu of a row, the row transform at dy is A - i sgn(dy) S, and
//   lambda(dx, dy) = sum_kx (cos(kx dx theta) - i sin(kx dx theta)) (A - i sgn(dy) S).

// half-plane points: the diamond |dx| + |dy| <= 4 (NDY = 4) or the 5 x 5 box (NDY = 2)
template <int NDY>
struct Half;
template <>
struct Half<4> {
  static constexpr int N = 21;
  __host__ __device__ static constexpr int dx(int h) { return h < 5 ? 0 : h < 12 ? 1 : h < 17 ? 2 : h < 20 ? 3 : 4; }
  __host__ __device__ static constexpr int dy(int h) {
    return h < 5 ? h : h < 12 ? h - 5 - 3 : h < 17 ? h - 12 - 2 : h < 20 ? h - 17 - 1 : 0;
  }
};
template <>
struct Half<2> {
  static constexpr int N = 13;
  __host__ __device__ static constexpr int dx(int h) { return h < 3 ? 0 : h < 8 ? 1 : 2; }
  __host__ __device__ static constexpr int dy(int h) { return h < 3 ? h : h < 8 ? h - 3 - 2 : h - 8 - 2; }
};

template <int NDY>
__global__ __launch_bounds__(256) void loop_rb_rowsum_kernel(const float *__restrict__ Y,
                                                             const double *__restrict__ tw, int Lf, int n_q,
                                                             int ch, double *__restrict__ lam_out) {
  using S = RB<NDY>;
  using H = Half<NDY>;
  constexpr int ROWS = S::ROWS;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  // threads cover whole groups of NQG coarse q: (group, alpha, (q in group, beta))
  const long long total = (long long)((n_q + NQG - 1) / NQG) * NQG * NA * NA;
  if (i >= total) return;
  // consecutive threads along (q within group, beta)
  const int col = (int)(i % NCOL);
  const int alpha = (int)((i / NCOL) % NA);
  const int g = (int)(i / ((long long)NCOL * NA));
  const int ql = col / NA;
  const int q = NQG * g + ql;
  if (q >= n_q) return;
  const int beta = col % NA;
  double zr[H::N], zi[H::N];
#pragma unroll
  for (int h = 0; h < H::N; ++h) zr[h] = zi[h] = 0.0;
  const float *Yg = Y + (size_t)g * Lf * ROWS * NCOL + (size_t)alpha * NCOL + col;
  for (int kx = 0; kx < Lf; ++kx) {
    const float *Yr = Yg + (size_t)kx * ROWS * NCOL;
    double v[2 * NDY + 1];
#pragma unroll
    for (int f = 0; f < 2 * NDY + 1; ++f) v[f] = (double)Yr[(size_t)f * NA * NCOL];
    double cx[NDY + 1], sx[NDY + 1];
    cx[0] = 1.0;
    sx[0] = 0.0;
#pragma unroll
    for (int dx = 1; dx <= NDY; ++dx) {
      const int jj = (int)(((long long)kx * dx) % Lf);
      cx[dx] = tw[2 * jj];
      sx[dx] = -tw[2 * jj + 1];
    }
#pragma unroll
    for (int h = 0; h < H::N; ++h) {
      const int dx = H::dx(h), dy = H::dy(h), ad = dy < 0 ? -dy : dy;
      const double A = v[ad];
      if (dy == 0) {
        zr[h] = fma(cx[dx], A, zr[h]);
        zi[h] = fma(-sx[dx], A, zi[h]);
      } else {
        const double Sg = dy > 0 ? v[NDY + ad] : -v[NDY + ad];
        zr[h] = fma(cx[dx], A, fma(-sx[dx], Sg, zr[h]));
        zi[h] = fma(-cx[dx], Sg, fma(-sx[dx], A, zi[h]));
      }
    }
  }
  // lam_out[q][h][alpha][beta] complex; ph: the imaginary coordinates beta
  // of the transposed X change sign
  const double sg = (ch == 1 && beta >= NO && ((beta - NO) & 1)) ? -1.0 : 1.0;
#pragma unroll
  for (int h = 0; h < H::N; ++h) {
    const size_t o = (((size_t)q * H::N + h) * NA + alpha) * NA + beta;
    lam_out[2 * o] = sg * zr[h];
    lam_out[2 * o + 1] = sg * zi[h];
  }
}

// real-basis coordinates of the matrix entry (a, c): one (diagonal) or two
// (real part, imaginary part times +-i) coordinates
__device__ inline int rb_coords(int a, int c, int *alpha, double *ci) {
  if (a == c) {
    alpha[0] = a;
    ci[0] = 0.0;
    return 1;
  }
  const int lo = a < c ? a : c, hi = a < c ? c : a;
  int p = 0;
  for (int x = 0; x < lo; ++x) p += NO - 1 - x;
  p += hi - lo - 1;
  alpha[0] = NO + 2 * p;
  alpha[1] = NO + 2 * p + 1;
  ci[0] = 0.0;
  ci[1] = a < c ? 1.0 : -1.0;  // coefficient of the second coordinate: i ci[1]
  return 2;
}

// compact[q][iD][(a b c d)] = 1/Nf sum E^alpha_ac E^beta_bd lambda^{alpha beta}(q, +-dR)
template <int NDY>
__global__ __launch_bounds__(256) void loop_rb_finalize_kernel(int n_q, int nD, const int *__restrict__ hmap,
                                                               double inv_nf, const double *__restrict__ lam,
                                                               double *__restrict__ compact) {
  using H = Half<NDY>;
  constexpr int NO2 = NO * NO, NO3 = NO2 * NO, NO4 = NO2 * NO2;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n_q * nD * NO4) return;
  const int tau = (int)(i % NO4);
  const int iD = (int)((i / NO4) % nD);
  const int q = (int)(i / ((long long)NO4 * nD));
  const int hm = hmap[iD], h = hm & 0xffff;
  const bool cj = (hm >> 16) != 0;  // the other half plane: lambda(-dR) = conj lambda(dR)
  const int a = tau / NO3, b = (tau / NO2) % NO, c = (tau / NO) % NO, d = tau % NO;
  int al[2], be[2];
  double ca[2], cb[2];
  const int na = rb_coords(a, c, al, ca), nb = rb_coords(b, d, be, cb);
  double sr = 0.0, si = 0.0;
  for (int x = 0; x < na; ++x)
    for (int y = 0; y < nb; ++y) {
      const size_t o = (((size_t)q * H::N + h) * NA + al[x]) * NA + be[y];
      const double lr = lam[2 * o], li = cj ? -lam[2 * o + 1] : lam[2 * o + 1];
      // coefficient (x ? i ca : 1) (y ? i cb : 1)
      if (x == 0 && y == 0) {
        sr += lr;
        si += li;
      } else if (x == 1 && y == 1) {
        const double f = -ca[1] * cb[1];
        sr += f * lr;
        si += f * li;
      } else {
        const double f = x == 1 ? ca[1] : cb[1];  // times i
        sr -= f * li;
        si += f * lr;
      }
    }
  compact[2 * i] = sr * inv_nf;
  compact[2 * i + 1] = si * inv_nf;
}

size_t loop_rb_rowbuf_floats(int ndy, int Lf) {
  const int rows = (2 * ndy + 1) * NA;
  return (size_t)Lf * rows * NCOL;  // per group of NQG coarse q
}

int loop_rb_half_points(int ndy, int *dx, int *dy) {
  if (ndy == 4) {
    for (int h = 0; h < Half<4>::N; ++h) {
      dx[h] = Half<4>::dx(h);
      dy[h] = Half<4>::dy(h);
    }
    return Half<4>::N;
  }
  if (ndy == 2) {
    for (int h = 0; h < Half<2>::N; ++h) {
      dx[h] = Half<2>::dx(h);
      dy[h] = Half<2>::dy(h);
    }
    return Half<2>::N;
  }
  return 0;
}

size_t loop_rb_apre_bytes(int ndy, int Lf, int pair) {
  const int mt = ndy == 4 ? RB<4>::MT : RB<2>::MT;
  const size_t ntk = (size_t)((pair ? Lf / 2 : Lf) + KT - 1) / KT;
  return (size_t)Lf * ntk * KS * mt * 2 * 64 * 16;
}

// the precomputed A operand of every kx row (once per context; band data and
// phases are those of the loop kernel: FP32, k-major; paired: the pair sums of
// the projectors)
hipError_t launch_loop_rb_apre(int ndy, int pair, const float *band, const float *pir, const float *phy, int Lf,
                               void *apre, hipStream_t st) {
  if (!band || !phy || !apre || (ndy != 2 && ndy != 4) || (pair && (!pir || Lf % 2))) return hipErrorInvalidValue;
  const int mt = ndy == 4 ? RB<4>::MT : RB<2>::MT;
  const long long n = (long long)Lf * (((pair ? Lf / 2 : Lf) + KT - 1) / KT) * KS * mt * 64;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (ndy == 4 && pair)
    hipLaunchKernelGGL((loop_rb_apre_kernel<4, true>), grid, dim3(256), 0, st, band, pir, phy, Lf, (u32x4 *)apre);
  else if (ndy == 4)
    hipLaunchKernelGGL((loop_rb_apre_kernel<4, false>), grid, dim3(256), 0, st, band, pir, phy, Lf, (u32x4 *)apre);
  else if (pair)
    hipLaunchKernelGGL((loop_rb_apre_kernel<2, true>), grid, dim3(256), 0, st, band, pir, phy, Lf, (u32x4 *)apre);
  else
    hipLaunchKernelGGL((loop_rb_apre_kernel<2, false>), grid, dim3(256), 0, st, band, pir, phy, Lf, (u32x4 *)apre);
  return hipGetLastError();
}

// pair sums of the projectors of bands (0, 1), (2, 3), (4, 5), summed in FP64
// (and rounded to FP32): pir[k][p][alpha] from the component-major band data
__global__ void pair_pi_kernel(int Nf, const double *__restrict__ band, float *__restrict__ pir,
                               double *__restrict__ pir64) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)Nf * 3 * NA) return;
  const int k = (int)(i / (3 * NA)), r = (int)(i % (3 * NA)), p = r / NA, alpha = r % NA;
  const double a = band[(size_t)(NO + 2 * p * NA + alpha) * Nf + k];
  const double b = band[(size_t)(NO + (2 * p + 1) * NA + alpha) * Nf + k];
  if (pir) pir[i] = (float)(a + b);
  if (pir64) pir64[i] = a + b;
}

hipError_t launch_pair_pi(int Nf, const double *band, float *pir, double *pir64, hipStream_t st) {
  if (!band || (!pir && !pir64) || Nf < 1) return hipErrorInvalidValue;
  const long long n = (long long)Nf * 3 * NA;
  hipLaunchKernelGGL(pair_pi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Nf, band, pir, pir64);
  return hipGetLastError();
}

// one channel, coarse q [q_first, q_first + n_q) (or the q_x rows of a.rows):
// the row buffers Y (ceil(n_q / 4) groups of loop_rb_rowbuf_floats), with the
// A operand apre of launch_loop_rb_apre (of the same pairing)
hipError_t launch_loop_rb(const LoopArgs &a, int ch, const void *apre, float *Y, hipStream_t st) {
  if (a.n_o != NO || !Y || !apre) return hipErrorInvalidValue;
  const float *band = (const float *)a.band, *kv = (const float *)a.kv;
  const float *cvp = (const float *)a.cv, *pir = a.pir;
  if (a.scheme == CUT_SHELL && !cvp) return hipErrorInvalidValue;
  if (a.pair && (!pir || a.Lf % 2)) return hipErrorInvalidValue;
  if (!(a.ndy == 4 && a.ndx == 5) && !(a.ndy == 2 && a.ndx == 3)) return hipErrorInvalidValue;
  const int n_groups = (a.n_q + NQG - 1) / NQG;
  const int kxr = a.kxr;  // kx rows per work item
  if (kxr < 1 || kxr > 8) return hipErrorInvalidValue;
  const int n_kxb = (a.Lf + kxr - 1) / kxr;
  const long long nblk = 8LL * n_groups * ((n_kxb + 7) / 8);
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  const float lam = (float)a.lam;
  const bf16x8 *ap = (const bf16x8 *)apre;
#define TUFRG_RB_LAUNCH(D, S, P)                                                                                   \
  hipLaunchKernelGGL((loop_rb_kernel<D, S, P>), dim3((unsigned)nblk), dim3(NTHR), 0, st, band, pir, kv, cvp, ap, \
                     a.Lq, a.n_ref, a.Lf, a.q_first, a.n_q, a.rows, ch, lam, a.deriv, n_groups, n_kxb, kxr, Y)
#define TUFRG_RB_SCHEMES(D, P)              \
  if (a.scheme == CUT_TEMPERATURE)          \
    TUFRG_RB_LAUNCH(D, CUT_TEMPERATURE, P); \
  else if (a.scheme == CUT_OMEGA)           \
    TUFRG_RB_LAUNCH(D, CUT_OMEGA, P);       \
  else if (a.scheme == CUT_SHELL)           \
    TUFRG_RB_LAUNCH(D, CUT_SHELL, P);       \
  else                                      \
    return hipErrorInvalidValue;
  if (a.ndy == 4 && a.pair) {
    TUFRG_RB_SCHEMES(4, true)
  } else if (a.ndy == 4) {
    TUFRG_RB_SCHEMES(4, false)
  } else if (a.pair) {
    TUFRG_RB_SCHEMES(2, true)
  } else {
    TUFRG_RB_SCHEMES(2, false)
  }
#undef TUFRG_RB_SCHEMES
#undef TUFRG_RB_LAUNCH
  return hipGetLastError();
}

// then the real-basis sums lamb ([n_q][half points][36][36] complex) and the
// compact loops at dst ([n_q][nD][n_o^4] complex); hmap[iD] = half-plane point
// of dlist[iD] (low 16 bits) and 1 << 16 where it is the reflected one
hipError_t launch_loop_rb_sums(const LoopArgs &a, const float *Y, double *lamb, const int *hmap, int nD,
                               double *dst, hipStream_t st) {
  if (!Y || !lamb || !hmap || !dst || a.n_ch != 1) return hipErrorInvalidValue;
  const int n_groups = (a.n_q + NQG - 1) / NQG;
  const long long nt = (long long)n_groups * NQG * NA * NA;
  const long long nf = (long long)a.n_q * nD * NO * NO * NO * NO;
  const double inv = 1.0 / ((double)a.Lf * a.Lf);
  if (a.ndy == 4) {
    hipLaunchKernelGGL(loop_rb_rowsum_kernel<4>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, Y, a.tw, a.Lf,
                       a.n_q, a.ch_first, lamb);
    hipLaunchKernelGGL(loop_rb_finalize_kernel<4>, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, a.n_q, nD,
                       hmap, inv, lamb, dst);
  } else if (a.ndy == 2) {
    hipLaunchKernelGGL(loop_rb_rowsum_kernel<2>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, Y, a.tw, a.Lf,
                       a.n_q, a.ch_first, lamb);
    hipLaunchKernelGGL(loop_rb_finalize_kernel<2>, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, a.n_q, nD,
                       hmap, inv, lamb, dst);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tufrg

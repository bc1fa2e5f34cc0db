// Form-factor projected orbital loops for NO > 2 spin-orbitals (hot path of
// multi-orbital models such as t2g with spin-orbit coupling).
//
// Same quantity as the two-orbital kernel (see k_loop.hip):
//   Lc(q)[dR][(a,b,c,d)] = 1/Nf sum_k e^{-ik.dR} M_q(k)[a,b,c,d],
//   M_q(k)[a,b,c,d] = sum_m Pi_m(k)_ac W_m(k)_bd,  W_m = sum_n L_mn X_n,
// with X_n = Pi_n(k') (pp, k' = q - k) or its transpose (ph, k' = k - q).
//
// Entry pairs.  Pi_m and W_m are Hermitian, so M[(c,d,a,b)] = conj M[(a,b,c,d)]
// and Lc[dR][(c,d,a,b)] = conj Lc[-dR][(a,b,c,d)].  A thread owns one pair of
// such entries (or a self-conjugate entry), listed by the host: it forms M for
// the first entry at every k and keeps its loop for every dR of the
// difference set D of the form factors; the partner follows at the end.
//
// Separable phases.  Over one kx row the thread accumulates S = sum M and, for
// dy = 1..NDY, A = sum cos(theta) M and B = sum -sin(theta) M with
// theta = 2 pi ky dy / Lf (table phy[ky][dy - 1], read by scalar loads), so that the row transform at +dy is A + iB and at
// -dy is A - iB.  At the end of the row Lc[(dx, dy)] += e^{-i kx dx} Y(dy) for
// every (dx, dy) in D.
//
// Staging.  Per tile of KT consecutive ky the workgroup writes to LDS the
// projectors Pi_m(k) as full complex NO x NO matrices, the packed X_n(k'), the
// loop kernels L_mn and then W_m(k) as full complex matrices, so that the
// inner loop reads one complex value of Pi and one of W per band.
//
// Kramers pairs (PAIR): when bands (0,1), (2,3), (4,5) are degenerate at every
// k, L_mn depends on the pairs only and the band sums group exactly into three
// bands with the pair sums of the projectors (energies and regulator values
// of the first band of each pair).
#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) c2 {
  T re, im;
};

// points (dx, dy) of the difference set: the 9-vector shell gives the 5 x 5
// box (R = 2), the 13-vector shell the diamond |dx| + |dy| <= 4 (R = 4)
template <int R>
struct Shape;
template <>
struct Shape<2> {
  static constexpr int N = 25;
  __device__ static constexpr int dx(int i) { return i / 5 - 2; }
  __device__ static constexpr int dy(int i) { return i % 5 - 2; }
};
template <>
struct Shape<4> {
  static constexpr int N = 41;
  __device__ static constexpr int row_len(int x) { return 2 * (4 - (x < 0 ? -x : x)) + 1; }
  __device__ static constexpr int row_start(int x) {
    int s = 0;
    for (int r = -4; r < x; ++r) s += row_len(r);
    return s;
  }
  __device__ static constexpr int dx(int i) {
    int x = -4;
    while (x < 4 && row_start(x + 1) <= i) ++x;
    return x;
  }
  __device__ static constexpr int dy(int i) { return i - row_start(dx(i)) - (row_len(dx(i)) - 1) / 2; }
};

// packed Hermitian NO x NO matrix: NO diagonal reals, then Re and Im of (lo, hi)
// for lo < hi in row-major order; slot -> (lo, hi) of an off-diagonal pair
template <int NO>
__device__ inline void pair_of(int p, int &lo, int &hi) {
  lo = 0;
  while (p >= NO - 1 - lo) {
    p -= NO - 1 - lo;
    ++lo;
  }
  hi = lo + 1 + p;
}

// writes packed value x of slot pl into the full complex matrix dst[NO][NO]
template <typename T, int NO>
__device__ inline void unpack_store(c2<T> *dst, int pl, T x) {
  if (pl < NO) {
    c2<T> v;
    v.re = x;
    v.im = T(0);
    dst[pl * NO + pl] = v;
    return;
  }
  const int q = pl - NO;
  int lo, hi;
  pair_of<NO>(q >> 1, lo, hi);
  if (q & 1) {
    dst[lo * NO + hi].im = x;
    dst[hi * NO + lo].im = -x;
  } else {
    dst[lo * NO + hi].re = x;
    dst[hi * NO + lo].re = x;
  }
}

}  // namespace

// One workgroup per (part, channel, q); part selects NTHR of the entry pairs.
template <typename T, int NO, int NDY, int SCHEME, int NTHR, int KT, bool PAIR>
__global__ __launch_bounds__(NTHR) void loop_gen_kernel(const T *__restrict__ band, const T *__restrict__ pir,
                                                        const T *__restrict__ kv, const T *__restrict__ cvp,
                                                        const double *__restrict__ tw, const T *__restrict__ phy,
                                                        const int *__restrict__ pairs,
                                                        int n_pairs, int Lq, int n_ref, int Lf, int nparts,
                                                        int q_first, int n_q, const int *__restrict__ rows,
                                                        int ch_first, int n_ch, int ndx_out,
                                                        T lam, int deriv, T *__restrict__ partial) {
  using SH = Shape<NDY>;
  constexpr int NPT = SH::N;
  constexpr int NO2 = NO * NO, NO4 = NO2 * NO2;
  constexpr int NB = PAIR ? NO / 2 : NO;  // bands summed (pairs)
  constexpr int PK = NB * NO2;      // packed reals of the summed bands' projectors at one k
  constexpr int NC = NO + NO * NO2; // band values per k-point: e_m, then the packed projectors
  constexpr bool SHELL = SCHEME == CUT_SHELL;
  // band m of the sums in the arrays of all bands (paired: the first of the pair)
  constexpr int MS = PAIR ? 2 : 1;
  // staged values per k-point: energies, packed projectors and regulator
  // values (and the shell factors a_m, b_m of the momentum-shell scheme)
  constexpr int NIT = NB + PK + NB + (SHELL ? 2 * NB : 0);
  const int tid = threadIdx.x;
  int w = blockIdx.x;
  const int part = w % nparts;
  w /= nparts;
  const int chrel = w % n_ch, qrel = w / n_ch;
  // coarse q: consecutive from q_first, or whole q_x rows from a list
  const int qi = rows ? rows[qrel / Lq] * Lq + qrel % Lq : q_first + qrel, ch = ch_first + chrel;
  const int qfx = (qi / Lq) * n_ref, qfy = (qi % Lq) * n_ref;
  const int pidx = part * NTHR + tid;
  const bool active = pidx < n_pairs;
  const int tau = active ? pairs[2 * pidx] : 0, taub = active ? pairs[2 * pidx + 1] : 0;
  const int xo = (tau / (NO * NO2)) * NO + (tau / NO) % NO;  // (a, c)
  const int yo = ((tau / NO2) % NO) * NO + tau % NO;        // (b, d)

  __shared__ c2<T> sP[KT][NB][NO2];  // Pi_m(k)
  __shared__ c2<T> sW[KT][NB][NO2];  // W_m(k)
  __shared__ T sX[KT][PK];           // X_n(k') packed
  __shared__ T sE[KT][2][NB];        // e at k and k'
  __shared__ T sK[KT][2][NB];        // regulator at k and k'
  __shared__ T sL[KT][NB][NB];
  __shared__ T sC[SHELL ? KT : 1][2][2 * NB];  // shell factors (a_m, b_m) at k and k'
  const T sg = (ch == 0) ? T(1) : T(-1);

  cx<T> Z[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) Z[i] = cmake(T(0), T(0));

  for (int kx = 0; kx < Lf; ++kx) {
    int kpx = (ch == 0) ? (qfx - kx) : (kx - qfx);
    kpx += kpx < 0 ? Lf : 0;
    cx<T> S = cmake(T(0), T(0)), A[NDY], B[NDY];
#pragma unroll
    for (int j = 0; j < NDY; ++j) A[j] = B[j] = cmake(T(0), T(0));
    for (int ky0 = 0; ky0 < Lf; ky0 += KT) {
      __syncthreads();
#pragma unroll 1
      for (int i = tid; i < KT * 2 * NIT; i += NTHR) {
        const int r = i % NIT, t2 = i / NIT;
        const int j = t2 >> 1, side = t2 & 1;
        const int ky = ky0 + j < Lf ? ky0 + j : Lf - 1;
        int kpy = (ch == 0) ? (qfy - ky) : (ky - qfy);
        kpy += kpy < 0 ? Lf : 0;
        const unsigned kk = side ? (unsigned)kpx * Lf + kpy : (unsigned)kx * Lf + ky;
        if (r < NB) {
          sE[j][side][r] = band[(size_t)kk * NC + MS * r];
        } else if (r < NB + PK) {
          const int p = r - NB, m = p / NO2, pl = p % NO2;
          T x = PAIR ? pir[(size_t)kk * PK + p] : band[(size_t)kk * NC + NO + p];
          if (side == 0) {
            unpack_store<T, NO>(&sP[j][m][0], pl, x);
          } else {
            // ph uses the transpose of Pi_n(k'): flip the imaginary parts
            if (ch == 1 && pl >= NO && ((pl - NO) & 1)) x = -x;
            sX[j][p] = x;
          }
        } else if (r < NB + PK + NB) {
          sK[j][side][r - NB - PK] = kv[(size_t)kk * NO + MS * (r - NB - PK)];
        } else if constexpr (SHELL) {
          const int c = r - 2 * NB - PK;  // (a_m, b_m) of summed band c / 2
          sC[j][side][c] = cvp[(size_t)kk * 2 * NO + 2 * MS * (c >> 1) + (c & 1)];
        }
      }
      __syncthreads();
      // loop kernels L_mn = sg * DD[K](e_m(k), -sg e_n(k'))
      if (tid < KT * NB * NB) {
        const int j = tid / (NB * NB), m = (tid / NB) % NB, n = tid % NB;
        const T x = sE[j][0][m], y = -sg * sE[j][1][n];
        T l = sg * divided_difference(x, y, sK[j][0][m], -sg * sK[j][1][n], lam, dd_scheme(SCHEME), deriv);
        // shell scheme: times a_m(k) b_n(k') + b_m(k) a_n(k')
        if constexpr (SHELL) l *= fma(sC[j][0][2 * m], sC[j][1][2 * n + 1], sC[j][0][2 * m + 1] * sC[j][1][2 * n]);
        sL[j][m][n] = l;
      }
      __syncthreads();
      // W_m = sum_n L_mn X_n, packed sums written as full complex matrices
#pragma unroll 1
      for (int i = tid; i < KT * PK; i += NTHR) {
        const int j = i / PK, mp = i % PK, m = mp / NO2, pl = mp % NO2;
        T acc = T(0);
#pragma unroll
        for (int n = 0; n < NB; ++n) acc = fma(sL[j][m][n], sX[j][n * NO2 + pl], acc);
        unpack_store<T, NO>(&sW[j][m][0], pl, acc);
      }
      __syncthreads();
      const int kt = min(KT, Lf - ky0);
      for (int j = 0; j < kt; ++j) {
        // the same for every lane: scalar loads
        const T *ph = phy + (size_t)(ky0 + j) * (2 * NDY);
        cx<T> M = cmake(T(0), T(0));
#pragma unroll
        for (int m = 0; m < NB; ++m) {
          const c2<T> P = sP[j][m][xo], Wv = sW[j][m][yo];
          cfma(M, cmake(P.re, P.im), cmake(Wv.re, Wv.im));
        }
        S.re += M.re;
        S.im += M.im;
#pragma unroll
        for (int dy = 0; dy < NDY; ++dy) {
          const T cs = ph[2 * dy], sn = ph[2 * dy + 1];
          A[dy].re = fma(cs, M.re, A[dy].re);
          A[dy].im = fma(cs, M.im, A[dy].im);
          B[dy].re = fma(sn, M.re, B[dy].re);
          B[dy].im = fma(sn, M.im, B[dy].im);
        }
      }
    }
    // row transform at +dy: A + iB, at -dy: A - iB; then the kx phase,
    // one |dx| at a time
#pragma unroll
    for (int adx = 0; adx <= NDY; ++adx) {
      const int jj = (kx * adx) % Lf;
      const cx<T> p = cmake((T)tw[2 * jj], (T)tw[2 * jj + 1]);
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int dx = SH::dx(i), dy = SH::dy(i);
        if ((dx < 0 ? -dx : dx) != adx) continue;
        cx<T> Yv;
        if (dy == 0) {
          Yv = S;
        } else {
          const cx<T> Av = A[(dy > 0 ? dy : -dy) - 1], Bv = B[(dy > 0 ? dy : -dy) - 1];
          Yv = dy > 0 ? cmake(Av.re - Bv.im, Av.im + Bv.re) : cmake(Av.re + Bv.im, Av.im - Bv.re);
        }
        cfma(Z[i], dx < 0 ? cmake(p.re, -p.im) : p, Yv);
      }
    }
  }
  if (!active) return;
  // partial[ch][q][dx][dy + NDY][tau] for dx >= 0; the partner entry from
  // Lc[dR][partner] = conj Lc[-dR][tau]
  const int ndy2 = 2 * NDY + 1;
  const size_t pbase = ((size_t)chrel * n_q + qrel) * (size_t)(ndx_out * ndy2 * NO4);
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int dx = SH::dx(i), dy = SH::dy(i);
    if (dx >= 0) {
      const size_t idx = pbase + (size_t)(dx * ndy2 + dy + NDY) * NO4 + tau;
      partial[2 * idx] = Z[i].re;
      partial[2 * idx + 1] = Z[i].im;
    }
    if (dx <= 0 && taub != tau) {
      const size_t idx = pbase + (size_t)(-dx * ndy2 - dy + NDY) * NO4 + taub;
      partial[2 * idx] = Z[i].re;
      partial[2 * idx + 1] = -Z[i].im;
    }
  }
}

template <typename T, int NDY>
static hipError_t launch_gen(const LoopArgs &a, hipStream_t st) {
  // FP32: every pair of a (q, channel) in one workgroup of 11 waves (three
  // per SIMD); FP64 needs twice the registers: workgroups of 6 waves
  constexpr bool f64 = sizeof(T) == 8;
  constexpr int NTHR = f64 ? 384 : 704, KT = f64 ? 8 : 16;
  if (a.ndx != NDY + 1) return hipErrorInvalidValue;
  const int NP = (a.n_pairs + NTHR - 1) / NTHR;
  dim3 grid(a.n_q * a.n_ch * NP), block(NTHR);
  const T *band = (const T *)a.band, *kv = (const T *)a.kv, *phy = (const T *)a.phy, *cvp = (const T *)a.cv;
  const T *pir = f64 ? (const T *)a.pir64 : (const T *)a.pir;
  if (a.scheme == CUT_SHELL && !cvp) return hipErrorInvalidValue;
  if (a.pair && !pir) return hipErrorInvalidValue;
#define TUFRG_GEN_LAUNCH(S, P)                                                                                   \
  hipLaunchKernelGGL((loop_gen_kernel<T, 6, NDY, S, NTHR, KT, P>), grid, block, 0, st, band, pir, kv, cvp, a.tw, \
                     phy, a.pairs, a.n_pairs, a.Lq, a.n_ref, a.Lf, NP, a.q_first, a.n_q, a.rows, a.ch_first,     \
                     a.n_ch, a.ndx, (T)a.lam, a.deriv, (T *)a.partial)
#define TUFRG_GEN_SCHEMES(P)               \
  if (a.scheme == CUT_TEMPERATURE)         \
    TUFRG_GEN_LAUNCH(CUT_TEMPERATURE, P);  \
  else if (a.scheme == CUT_OMEGA)          \
    TUFRG_GEN_LAUNCH(CUT_OMEGA, P);        \
  else if (a.scheme == CUT_SHELL)          \
    TUFRG_GEN_LAUNCH(CUT_SHELL, P);        \
  else                                     \
    return hipErrorInvalidValue;
  if (a.pair) {
    TUFRG_GEN_SCHEMES(true)
  } else {
    TUFRG_GEN_SCHEMES(false)
  }
#undef TUFRG_GEN_SCHEMES
#undef TUFRG_GEN_LAUNCH
  return hipGetLastError();
}

hipError_t launch_loop_gen(const LoopArgs &a, hipStream_t st) {
  if (a.n_o != 6 || !a.pairs || a.n_pairs <= 0) return hipErrorInvalidValue;
  const bool f64 = (a.prec == 0);
  if (a.ndx == 5 && a.ndy == 4) return f64 ? launch_gen<double, 4>(a, st) : launch_gen<float, 4>(a, st);
  if (a.ndx == 3 && a.ndy == 2) return f64 ? launch_gen<double, 2>(a, st) : launch_gen<float, 2>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace tufrg

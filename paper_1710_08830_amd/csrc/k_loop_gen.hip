// Form-factor projected orbital loops for NO > 2 spin-orbitals (hot path of
// multi-orbital models such as t2g with spin-orbit coupling).
//
// Same quantity as the two-orbital kernel (see k_loop.hip):
//   Lc(q)[dR][(a,b,c,d)] = 1/Nf sum_k e^{-ik.dR} M_q(k)[a,b,c,d],
//   M_q(k)[a,b,c,d] = sum_m Pi_m(k)_ac W_m(k)_bd,  W_m = sum_n L_mn X_n,
// with X_n = Pi_n(k') (pp, k' = q - k) or its transpose (ph, k' = k - q).
//
// With NO^4 = 1296 entries per (q, channel) the entries are spread over the
// threads of a workgroup (one entry per thread, NPART workgroups per
// (q, channel)).  Per tile of KT consecutive ky the workgroup stages in LDS the
// band projectors Pi_m(k) and W_m(k) (both Hermitian, packed as NO^2 reals per
// band), computed once per tile from the band data at k and k'.  Each thread
// then forms its entry of M and accumulates Y[dy] = sum_ky e^{-i ky dy} M over
// the kx row; at the end of the row Z[dx][dy] += e^{-i kx dx} Y[dy] for dx >= 0
// (dx < 0 follows from hermiticity in the finalising kernel).
#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {

// offset of entry (a, c) in a packed Hermitian NO x NO matrix and the sign of
// its imaginary part: diagonal a -> a; a < c -> NO + 2 p(a, c) (Re), +1 (Im)
template <int NO>
__device__ inline void herm_slot(int a, int c, int &re, int &im, float &imsign) {
  if (a == c) {
    re = a;
    im = -1;
    imsign = 0.f;
    return;
  }
  const int lo = a < c ? a : c, hi = a < c ? c : a;
  int p = 0;
  for (int x = 0; x < lo; ++x) p += NO - 1 - x;
  p += hi - lo - 1;
  re = NO + 2 * p;
  im = re + 1;
  imsign = (a < c) ? 1.f : -1.f;
}

}  // namespace

template <typename T, int NO, int NDX, int NDY, int SCHEME, int NTHR, int KT>
__global__ __launch_bounds__(NTHR) void loop_gen_kernel(const T *__restrict__ band, const T *__restrict__ kv,
                                                        const double *__restrict__ tw, int Lq, int n_ref, int Lf,
                                                        int nparts_tau, int q_first, int n_q, int ch_first,
                                                        int n_ch, T lam, int deriv, double *__restrict__ partial) {
  constexpr int NO2 = NO * NO, NO4 = NO2 * NO2, NDY2 = 2 * NDY + 1;
  constexpr int PK = NO * NO2;  // packed reals of all bands' projectors at one k
  constexpr int NC = NO + PK;   // band values per k-point: e_m, then the packed projectors
  const int tid = threadIdx.x;
  int w = blockIdx.x;
  const int part = w % nparts_tau;
  w /= nparts_tau;
  const int chrel = w % n_ch, qrel = w / n_ch;
  const int qi = q_first + qrel, ch = ch_first + chrel;
  const int qfx = (qi / Lq) * n_ref, qfy = (qi % Lq) * n_ref;
  const int per_part = (NO4 + nparts_tau - 1) / nparts_tau;
  const int tau = part * per_part + tid;
  const bool active = (tid < per_part) && (tau < NO4);
  const int tt = active ? tau : 0;
  const int a = tt / (NO * NO2), b = (tt / NO2) % NO, c = (tt / NO) % NO, d = tt % NO;
  int pre, pim, wre, wim;
  float psg, wsg;
  herm_slot<NO>(a, c, pre, pim, psg);
  herm_slot<NO>(b, d, wre, wim, wsg);

  __shared__ T sP[KT][PK];     // Pi_m(k) packed
  __shared__ T sW[KT][PK];     // W_m(k) packed
  __shared__ T sX[KT][PK];     // X_n(k') packed
  __shared__ T sE[KT][2][NO];  // e at k and k'
  __shared__ T sK[KT][2][NO];  // regulator at k and k'
  __shared__ T sL[KT][NO][NO];
  __shared__ T sPh[KT][NDY2][2];

  cx<T> Z[NDX][NDY2];
#pragma unroll
  for (int i = 0; i < NDX; ++i)
#pragma unroll
    for (int j = 0; j < NDY2; ++j) Z[i][j] = cmake(T(0), T(0));
  const T sg = (ch == 0) ? T(1) : T(-1);

  for (int kx = 0; kx < Lf; ++kx) {
    int kpx = (ch == 0) ? (qfx - kx) : (kx - qfx);
    kpx = ((kpx % Lf) + Lf) % Lf;
    cx<T> Y[NDY2];
#pragma unroll
    for (int j = 0; j < NDY2; ++j) Y[j] = cmake(T(0), T(0));
    for (int ky0 = 0; ky0 < Lf; ky0 += KT) {
      __syncthreads();
      // stage band data of the tile: per k-point NC contiguous values (k-major layout)
      for (int i = tid; i < KT * 2 * (NC + NO); i += NTHR) {
        const int r = i % (NC + NO), t2 = i / (NC + NO);
        const int side = t2 & 1, j = t2 >> 1;
        const int ky = ky0 + j < Lf ? ky0 + j : Lf - 1;
        int kpy = (ch == 0) ? (qfy - ky) : (ky - qfy);
        kpy = ((kpy % Lf) + Lf) % Lf;
        const unsigned kk = side ? (unsigned)kpx * Lf + kpy : (unsigned)kx * Lf + ky;
        if (r < NO) {
          sE[j][side][r] = band[(size_t)kk * NC + r];
        } else if (r < NC) {
          const int p = r - NO;
          T x = band[(size_t)kk * NC + r];
          if (side == 0) {
            sP[j][p] = x;
          } else {
            // ph uses the transpose of Pi_n(k'): flip the imaginary parts
            const int pl = p % NO2;
            if (ch == 1 && pl >= NO && ((pl - NO) & 1)) x = -x;
            sX[j][p] = x;
          }
        } else {
          sK[j][side][r - NC] = kv[(size_t)kk * NO + (r - NC)];
        }
      }
      for (int i = tid; i < KT * NDY2; i += NTHR) {
        const int j = i / NDY2, dyi = i % NDY2;
        int jj = (int)(((long long)(ky0 + j) * (dyi - NDY)) % Lf);
        if (jj < 0) jj += Lf;
        sPh[j][dyi][0] = (T)tw[2 * jj];
        sPh[j][dyi][1] = (T)tw[2 * jj + 1];
      }
      __syncthreads();
      // loop kernels L_mn = sg * DD[K](e_m(k), -sg e_n(k'))
      for (int i = tid; i < KT * NO2; i += NTHR) {
        const int j = i / NO2, m = (i / NO) % NO, n = i % NO;
        const T x = sE[j][0][m], y = -sg * sE[j][1][n];
        sL[j][m][n] = sg * divided_difference(x, y, sK[j][0][m], -sg * sK[j][1][n], lam, SCHEME, deriv);
      }
      __syncthreads();
      // W_m = sum_n L_mn X_n (packed)
      for (int i = tid; i < KT * PK; i += NTHR) {
        const int j = i / PK, m = (i / NO2) % NO, p = i % NO2;
        T s = T(0);
#pragma unroll
        for (int n = 0; n < NO; ++n) s = fma(sL[j][m][n], sX[j][n * NO2 + p], s);
        sW[j][m * NO2 + p] = s;
      }
      __syncthreads();
      const int kt = min(KT, Lf - ky0);
      for (int j = 0; j < kt; ++j) {
        cx<T> M = cmake(T(0), T(0));
#pragma unroll
        for (int m = 0; m < NO; ++m) {
          const cx<T> P = cmake(sP[j][m * NO2 + pre], pim >= 0 ? (T)psg * sP[j][m * NO2 + pim] : T(0));
          const cx<T> W = cmake(sW[j][m * NO2 + wre], wim >= 0 ? (T)wsg * sW[j][m * NO2 + wim] : T(0));
          cfma(M, P, W);
        }
#pragma unroll
        for (int dyi = 0; dyi < NDY2; ++dyi) cfma(Y[dyi], cmake(sPh[j][dyi][0], sPh[j][dyi][1]), M);
      }
    }
    // kx phases for dx >= 0
#pragma unroll
    for (int dx = 0; dx < NDX; ++dx) {
      const int jj = (kx * dx) % Lf;
      const cx<T> p = cmake((T)tw[2 * jj], (T)tw[2 * jj + 1]);
#pragma unroll
      for (int dyi = 0; dyi < NDY2; ++dyi) cfma(Z[dx][dyi], p, Y[dyi]);
    }
  }
  if (!active) return;
  const size_t pbase = ((size_t)chrel * n_q + qrel) * (size_t)(NDX * NDY2 * NO4);
#pragma unroll
  for (int dx = 0; dx < NDX; ++dx)
#pragma unroll
    for (int dyi = 0; dyi < NDY2; ++dyi) {
      const size_t idx = pbase + (size_t)(dx * NDY2 + dyi) * NO4 + tau;
      partial[2 * idx] = (double)Z[dx][dyi].re;
      partial[2 * idx + 1] = (double)Z[dx][dyi].im;
    }
}

template <typename T, int NDX, int NDY>
static hipError_t launch_gen(const LoopArgs &a, hipStream_t st) {
  // 1296 entries per (q, channel): 3 workgroups of 432 (7 waves); the FP64
  // 5 x 9 phase box needs the whole register file of a wave: 6 x 216 (4 waves)
  constexpr bool big = sizeof(T) == 8 && NDX > 3;
  constexpr int NTHR = big ? 256 : 448, KT = 8, NP = big ? 6 : 3;
  dim3 grid(a.n_q * a.n_ch * NP), block(NTHR);
  const T *band = (const T *)a.band, *kv = (const T *)a.kv;
  if (a.scheme == CUT_TEMPERATURE)
    hipLaunchKernelGGL((loop_gen_kernel<T, 6, NDX, NDY, CUT_TEMPERATURE, NTHR, KT>), grid, block, 0, st, band, kv,
                       a.tw, a.Lq, a.n_ref, a.Lf, NP, a.q_first, a.n_q, a.ch_first, a.n_ch, (T)a.lam, a.deriv,
                       a.partial);
  else
    hipLaunchKernelGGL((loop_gen_kernel<T, 6, NDX, NDY, CUT_OMEGA, NTHR, KT>), grid, block, 0, st, band, kv, a.tw,
                       a.Lq, a.n_ref, a.Lf, NP, a.q_first, a.n_q, a.ch_first, a.n_ch, (T)a.lam, a.deriv, a.partial);
  return hipGetLastError();
}

hipError_t launch_loop_gen(const LoopArgs &a, hipStream_t st) {
  if (a.n_o != 6) return hipErrorInvalidValue;
  const bool f64 = (a.prec == 0);
  if (a.ndx == 5 && a.ndy == 4) return f64 ? launch_gen<double, 5, 4>(a, st) : launch_gen<float, 5, 4>(a, st);
  if (a.ndx == 3 && a.ndy == 2) return f64 ? launch_gen<double, 3, 2>(a, st) : launch_gen<float, 3, 2>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace tufrg

// SU(2)-reduced flow of one orbital per site (spin-rotation invariant): the
// spinful exchange propagators carry two spin structures,
//   P = p d13 d24 - p^x d14 d23,  p^x^{RR'}(s) = e^{is.R'} p^{R,-R'}(s),
//   C = c d13 d24 - d d14 d23,
// so three n_ff x n_ff functions p, c, d per q carry the state (Sec. 2
// channel definitions, Sec. 3.1 matrix RGE with spin-independent loops).  The
// reduced equations (the paper cites them without printing them) are
//   dp = -(a~ Lpp a~x + a~x Lpp a~),
//   dc = 2 (2 c~ Lph c~ - c~ Lph d~ - d~ Lph c~),
//   dd = -2 d~ Lph d~,
// with a~ = p + v + PC(c) + PD(d), c~ = c + v + CP(p) + CD(d),
// d~ = d + v + CP(p^x) + CD(c) from the scalar cross projections of Sec. 3.3
// (v the onsite coefficient of d13 d24 - d14 d23).
//   loop1_kernel       the one-band loops Lc[ch][q][dR], FP64
//   su2_exch_kernel    X -> X^x
//   su2_gather_kernel  the rho-space gathers of a~, c~, d~
//   su2_bundle_kernel  dp (pp channel) or dc, dd (ph channel) per q
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

// part[ch - ch_first][q - q_first][kx chunk][iD] = sum over the kx rows of the
// chunk of e^{-ik.dR_iD} L(e(k), e(k')) (k' = q - k for pp, k - q for ph): per
// kx row the ky sums with the phases of |dy| <= 4 (cos and sin parts), then
// the kx phases per dR; one workgroup per (q, channel, kx chunk), its threads
// over ky (one wave per 64 ky, at most four)
template <int NDP>
__global__ __launch_bounds__(256) void loop1_kernel(int Lq, int n_ref, int Lf, int nD, const int *__restrict__ dlist,
                                                    const double *__restrict__ e, const double *__restrict__ kv,
                                                    const double *__restrict__ tw, double lam, int scheme, int deriv,
                                                    int ch_first, int q_first, int n_q, int nkxc, int kxper,
                                                    double *__restrict__ part) {
  __shared__ double red[4][NDP][2];
  const int qrel = blockIdx.x, chrel = blockIdx.y, kxc = blockIdx.z, ch = ch_first + chrel;
  const int q = q_first + qrel;
  const int qfx = (q / Lq) * n_ref, qfy = (q % Lq) * n_ref;
  const double sg = ch == 0 ? 1.0 : -1.0;
  const int tid = threadIdx.x, nthr = blockDim.x;
  double zr[NDP], zi[NDP];
#pragma unroll
  for (int i = 0; i < NDP; ++i) zr[i] = zi[i] = 0.0;
  const int x1 = min(Lf, (kxc + 1) * kxper);
  for (int kx = kxc * kxper; kx < x1; ++kx) {
    double A[5], S[5];
#pragma unroll
    for (int y = 0; y < 5; ++y) A[y] = S[y] = 0.0;
    int kpx = ch == 0 ? qfx - kx : kx - qfx;
    kpx += kpx < 0 ? Lf : 0;
    for (int ky = tid; ky < Lf; ky += nthr) {
      int kpy = ch == 0 ? qfy - ky : ky - qfy;
      kpy += kpy < 0 ? Lf : 0;
      const size_t k = (size_t)kx * Lf + ky, kp = (size_t)kpx * Lf + kpy;
      const double l = sg * divided_difference(e[k], -sg * e[kp], kv[k], -sg * kv[kp], lam, scheme, deriv);
      A[0] += l;
#pragma unroll
      for (int y = 1; y < 5; ++y) {
        const int j = (int)(((long long)ky * y) % Lf);
        A[y] = fma(tw[2 * j], l, A[y]);       // cos
        S[y] = fma(-tw[2 * j + 1], l, S[y]);  // sin
      }
    }
    // row value at dy: sum_ky e^{-i ky dy theta} l = A - i sgn(dy) S
#pragma unroll
    for (int i = 0; i < NDP; ++i)
      if (i < nD) {
        const int dx = dlist[2 * i], dy = dlist[2 * i + 1], ay = dy < 0 ? -dy : dy;
        const double vr = A[ay], vi = dy > 0 ? -S[ay] : (dy < 0 ? S[ay] : 0.0);
        int j = (int)(((long long)kx * dx) % Lf);
        j += j < 0 ? Lf : 0;
        const double pr = tw[2 * j], pi = tw[2 * j + 1];  // e^{-i kx dx theta}
        zr[i] = fma(pr, vr, fma(-pi, vi, zr[i]));
        zi[i] = fma(pr, vi, fma(pi, vr, zi[i]));
      }
  }
  const int w = tid >> 6, lane = tid & 63, nw = (nthr + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NDP; ++i) {
    const double a = wave_sum(zr[i]), b = wave_sum(zi[i]);
    if (lane == 0 && i < nD) {
      red[w][i][0] = a;
      red[w][i][1] = b;
    }
  }
  __syncthreads();
  if (tid < nD) {
    double a = 0.0, b = 0.0;
    for (int v = 0; v < nw; ++v) {
      a += red[v][tid][0];
      b += red[v][tid][1];
    }
    const size_t o = (((size_t)chrel * n_q + qrel) * nkxc + kxc) * nD + tid;
    part[2 * o] = a;
    part[2 * o + 1] = b;
  }
}

// out[ch][q][iD] = 1/Nf sum over the kx chunks in order
__global__ void loop1_reduce_kernel(long long n, int nkxc, int nD, double inv_nf, const double2 *__restrict__ part,
                                    double2 *__restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long cq = i / nD;
  const int iD = (int)(i - cq * nD);
  double a = 0.0, b = 0.0;
  for (int c = 0; c < nkxc; ++c) {
    const double2 v = part[(cq * nkxc + c) * nD + iD];
    a += v.x;
    b += v.y;
  }
  out[i] = make_double2(a * inv_nf, b * inv_nf);
}

size_t loop1_partial_doubles(int n_q, int nD, int nkxc) { return 2 * 2 * (size_t)n_q * nkxc * nD; }

hipError_t launch_loop1(int Lq, int n_ref, int nD, const int *dlist, const double *e, const double *kv,
                        const double *tw, double lam, int scheme, int deriv, int ch_first, int n_ch, int q_first,
                        int n_q, int nkxc, double *part, double *out, hipStream_t st) {
  const int Lf = Lq * n_ref;
  if (n_q < 1 || n_ch < 1 || n_ch > 2 || scheme == CUT_SHELL || nkxc < 1 || !part) return hipErrorInvalidValue;
  const int kxper = (Lf + nkxc - 1) / nkxc;
  nkxc = (Lf + kxper - 1) / kxper;
  const double inv = 1.0 / ((double)Lf * Lf);
  const dim3 grid((unsigned)n_q, (unsigned)n_ch, (unsigned)nkxc);
  const int nthr = std::min(256, ((Lf + 63) / 64) * 64);
#define TUFRG_L1(N)                                                                                                 \
  hipLaunchKernelGGL(loop1_kernel<N>, grid, dim3(nthr), 0, st, Lq, n_ref, Lf, nD, dlist, e, kv, tw, lam, scheme, \
                     deriv, ch_first, q_first, n_q, nkxc, kxper, part)
  if (nD <= 13)
    TUFRG_L1(13);
  else if (nD <= 25)
    TUFRG_L1(25);
  else if (nD <= 41)
    TUFRG_L1(41);
  else
    return hipErrorInvalidValue;
#undef TUFRG_L1
  const long long n = (long long)n_ch * n_q * nD;
  hipLaunchKernelGGL(loop1_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, nkxc, nD, inv,
                     (const double2 *)part, (double2 *)out);
  return hipGetLastError();
}

// Xx[q][i][j] = e^{iq.R_j} X[q][i][neg(j)], neg(j) the index of -R_j
__global__ void su2_exch_kernel(int n_ff, int Nq, int Lq, const int *__restrict__ ff, const int *__restrict__ fneg,
                                const double2 *__restrict__ twq, const double2 *__restrict__ X,
                                double2 *__restrict__ Xx) {
  const long long n = (long long)Nq * n_ff * n_ff;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(i % n_ff), r = (int)((i / n_ff) % n_ff);
    const int q = (int)(i / ((long long)n_ff * n_ff));
    int ph = ((q / Lq) * ff[2 * j] + (q % Lq) * ff[2 * j + 1]) % Lq;
    ph += ph < 0 ? Lq : 0;
    const double2 x = X[((long long)q * n_ff + r) * n_ff + fneg[j]], t = twq[ph];
    Xx[i] = make_double2(t.x * x.x - t.y * x.y, t.x * x.y + t.y * x.x);
  }
}

hipError_t launch_su2_exch(int n_ff, int Nq, int Lq, const int *ff, const int *fneg, const double *twq,
                           const double *X, double *Xx, hipStream_t st) {
  const long long n = (long long)Nq * n_ff * n_ff;
  const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(su2_exch_kernel, dim3(blocks), dim3(256), 0, st, n_ff, Nq, Lq, ff, fneg, (const double2 *)twq,
                     (const double2 *)X, (double2 *)Xx);
  return hipGetLastError();
}

// G[w][iD][i][j] for w = a~, c~, d~ from the rho-space coefficients
// rA = (p, c)(rho) and rB = (p^x, d)(rho), each [2][nD][B][B]:
//   a~: c(rho)[R+rho, R'-rho]  + d(rho-R')[R+rho-R', -rho]
//   c~: p(rho)[R+rho, R'-rho]  + d(-R')[R-R'+rho, rho]
//   d~: px(rho)[R+rho, R'-rho] + c(-R')[R-R'+rho, rho]
// (terms whose labels leave S, or whose coefficient argument leaves D, dropped)
__global__ void su2_gather_kernel(int B, int nD, const int *__restrict__ ff, const int *__restrict__ dlist,
                                  const int *__restrict__ ffgrid, const int *__restrict__ dgrid,
                                  const double2 *__restrict__ rA, const double2 *__restrict__ rB,
                                  double2 *__restrict__ G) {
  const long long BB = (long long)B * B;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3LL * nD * BB) return;
  const int col = (int)(i % B), row = (int)((i / B) % B), iD = (int)((i / BB) % nD), w = (int)(i / (BB * nD));
  auto fidx = [&](int x, int y) -> int {
    if (x < -8 || x > 8 || y < -8 || y > 8) return -1;
    return ffgrid[(x + 8) * 17 + (y + 8)];
  };
  auto didx = [&](int x, int y) -> int {
    if (x < -8 || x > 8 || y < -8 || y > 8) return -1;
    return dgrid[(x + 8) * 17 + (y + 8)];
  };
  const int Rx = ff[2 * row], Ry = ff[2 * row + 1], Sx = ff[2 * col], Sy = ff[2 * col + 1];
  const int px = dlist[2 * iD], py = dlist[2 * iD + 1];
  const double2 *p = rA, *c = rA + nD * BB, *pxr = rB, *d = rB + nD * BB;
  double gr = 0.0, gi = 0.0;
  const int A = fidx(Rx + px, Ry + py), Bc = fidx(Sx - px, Sy - py);
  if (A >= 0 && Bc >= 0) {
    const double2 v = (w == 0 ? c : w == 1 ? p : pxr)[(long long)iD * BB + (long long)A * B + Bc];
    gr += v.x;
    gi += v.y;
  }
  if (w == 0) {
    const int A2 = fidx(Rx + px - Sx, Ry + py - Sy), B2 = fidx(-px, -py), D2 = didx(px - Sx, py - Sy);
    if (A2 >= 0 && B2 >= 0 && D2 >= 0) {
      const double2 v = d[(long long)D2 * BB + (long long)A2 * B + B2];
      gr += v.x;
      gi += v.y;
    }
  } else {
    const int A4 = fidx(Rx - Sx + px, Ry - Sy + py), B4 = fidx(px, py), D4 = didx(-Sx, -Sy);
    if (A4 >= 0 && B4 >= 0 && D4 >= 0) {
      const double2 v = (w == 1 ? d : c)[(long long)D4 * BB + (long long)A4 * B + B4];
      gr += v.x;
      gi += v.y;
    }
  }
  G[i] = make_double2(gr, gi);
}

hipError_t launch_su2_gather(int B, int nD, const int *ff, const int *dlist, const int *ffgrid, const int *dgrid,
                             const double *rA, const double *rB, double *G, hipStream_t st) {
  const long long n = 3LL * nD * B * B;
  hipLaunchKernelGGL(su2_gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, nD, ff, dlist, ffgrid,
                     dgrid, (const double2 *)rA, (const double2 *)rB, (double2 *)G);
  return hipGetLastError();
}

// per q: channel 0: dp = f (-(X1 T1 + X2 T2)), T1 = L X2, T2 = L X1 with
// (X1, X2) = (a~, a~x), L = Lpp; channel 1: (X1, X2) = (c~, d~), L = Lph,
// U1 = L X1, U2 = L X2, dc = f 2 (2 X1 U1 - X1 U2 - X2 U1), dd = f (-2 X2 U2);
// L expanded from its compact form (didx: dR index of (R1, R2)); LDS holds
// X1, X2, L and the two products (5 B^2 complex)
__global__ __launch_bounds__(256) void su2_bundle_kernel(int B, int Nq, int nD, const int *__restrict__ didx,
                                                         const double2 *__restrict__ Lc,
                                                         const double2 *__restrict__ Va,
                                                         const double2 *__restrict__ Vax,
                                                         const double2 *__restrict__ Vc,
                                                         const double2 *__restrict__ Vd, double f,
                                                         double2 *__restrict__ dp, double2 *__restrict__ dc,
                                                         double2 *__restrict__ dd) {
  extern __shared__ double2 sm[];
  const int BB = B * B;
  double2 *X1 = sm, *X2 = sm + BB, *L = sm + 2 * BB, *T1 = sm + 3 * BB, *T2 = sm + 4 * BB;
  const int q = blockIdx.x, ch = blockIdx.y, tid = threadIdx.x;
  const size_t off = (size_t)q * BB;
  const double2 *S1 = ch == 0 ? Va : Vc, *S2 = ch == 0 ? Vax : Vd;
  const double2 *Lq = Lc + ((size_t)ch * Nq + q) * nD;
  for (int i = tid; i < BB; i += blockDim.x) {
    X1[i] = S1[off + i];
    X2[i] = S2[off + i];
    L[i] = Lq[didx[i]];
  }
  __syncthreads();
  auto mm = [&](const double2 *A, const double2 *Bm, int i, int j) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k < B; ++k) {
      const double2 a = A[i * B + k], b = Bm[k * B + j];
      re = fma(a.x, b.x, fma(-a.y, b.y, re));
      im = fma(a.x, b.y, fma(a.y, b.x, im));
    }
    return make_double2(re, im);
  };
  // ch 0: T1 = L X2, T2 = L X1;  ch 1: T1 = L X1 (U1), T2 = L X2 (U2)
  for (int e = tid; e < BB; e += blockDim.x) {
    const int i = e / B, j = e - (e / B) * B;
    T1[e] = mm(L, ch == 0 ? X2 : X1, i, j);
    T2[e] = mm(L, ch == 0 ? X1 : X2, i, j);
  }
  __syncthreads();
  for (int e = tid; e < BB; e += blockDim.x) {
    const int i = e / B, j = e - (e / B) * B;
    if (ch == 0) {
      const double2 u = mm(X1, T1, i, j), v = mm(X2, T2, i, j);
      dp[off + e] = make_double2(-f * (u.x + v.x), -f * (u.y + v.y));
    } else {
      const double2 a = mm(X1, T1, i, j), b = mm(X1, T2, i, j), c2 = mm(X2, T1, i, j), g = mm(X2, T2, i, j);
      dc[off + e] = make_double2(2.0 * f * (2.0 * a.x - b.x - c2.x), 2.0 * f * (2.0 * a.y - b.y - c2.y));
      dd[off + e] = make_double2(-2.0 * f * g.x, -2.0 * f * g.y);
    }
  }
}

hipError_t launch_su2_bundle(int B, int Nq, int nD, const int *didx, const double *Lc, const double *Va,
                             const double *Vax, const double *Vc, const double *Vd, double f, double *dp, double *dc,
                             double *dd, hipStream_t st) {
  if (B < 1 || B > 25) return hipErrorInvalidValue;
  const size_t lds = 5 * (size_t)B * B * sizeof(double2);
  hipLaunchKernelGGL(su2_bundle_kernel, dim3((unsigned)Nq, 2), dim3(256), lds, st, B, Nq, nD, didx,
                     (const double2 *)Lc, (const double2 *)Va, (const double2 *)Vax, (const double2 *)Vc,
                     (const double2 *)Vd, f, (double2 *)dp, (double2 *)dc, (double2 *)dd);
  return hipGetLastError();
}

}  // namespace tufrg

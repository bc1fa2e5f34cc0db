// Truncated-unity cross projections (hot path, HBM-bound).
//
// Matrix layouts (B = n_ff n_o^2, flat index r n_o^2 + a n_o + b):
//   P[q][(R,a,b),(R',c,d)] = P^{RR'}_{a b d c}(q),  C[q][(R,a,b),(R',c,d)] = C^{RR'}_{a d b c}(q).
// The projections of the paper's Sec. 3.3 read, in these layouts and with
// X(rho) = 1/Nq sum_q e^{i q.rho} X(q):
//   P[V^C](s)[(R,a,b),(R',c,d)] =  sum_rho e^{is.rho} C(rho)[(R+rho,a,d),(R'-rho,c,b)]
//   P[V^D](s)[(R,a,b),(R',c,d)] = -sum_rho e^{is.rho} C(rho-R')[(R+rho-R',a,c),(-rho,d,b)]
//   C[V^P](u)[(R,a,b),(R',c,d)] =  sum_rho e^{iu.rho} P(rho)[(R+rho,a,d),(R'-rho,c,b)]
//   C[V^D](u)[(R,a,b),(R',c,d)] = -sum_rho e^{iu.rho} C(-R')[(R-R'+rho,a,c),(rho,b,d)]
// (the P[V^D] line substitutes rho = R' + R'' in the paper's form, which carries
// an extra e^{is.R'}), every term whose form-factor labels leave S being dropped.
// So each projected vertex is X(q) + X[V0] + sum_rho e^{iq.rho} G_X(rho), with
// G_X gathered once per evaluation in rho-space:
//   ft             X(q) -> X(rho)   (HBM read of both states)
//   gather_kernel  X(rho) -> G_P(rho), G_C(rho)
//   assemble       G(rho) -> VP(q), VC(q)  (HBM read of the states, write of V)
// On the q-mesh q = 2 pi (qx, qy) / Lq the phase factorises,
// e^{iq.rho} = e^{2 pi i qx rho_x / Lq} e^{2 pi i qy rho_y / Lq}, and rho_y takes
// at most nine values y_s over D.  Both transforms therefore run in two
// streaming stages through a small intermediate M [rows][2][ny][B^2] (about
// four times fewer operations than the direct sum over q and rho, and few
// registers per thread, so that many loads are in flight):
//   ft:       M(qx, s) = sum_qy e^{2 pi i qy y_s / Lq} X(qx, qy);
//             X(rho) += sum_qx e^{2 pi i qx rho_x / Lq} M(qx, s(rho))
//   assemble: M(qx, s) = sum_{rho: s(rho) = s} e^{2 pi i qx rho_x / Lq} G(rho);
//             VX(qx, qy) = X + X[V0] + sum_s e^{2 pi i qy y_s / Lq} M(qx, s)
// for blocks of qx rows that fit the workspace.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tufrg {

constexpr int NYMAX = 9;
constexpr int RMAX = 16;  // qx rows per pass of the assembly's first stage

// M[r][w][s][e] = sum_qy e^{2 pi i qy y_s / Lq} X_w(x0 + r, qy)[e]; phy [Lq][ny]
__global__ __launch_bounds__(256) void ft_rows_kernel(int BB, int Lq, int ny, int x0, const double *__restrict__ phy,
                                                      const double *__restrict__ P, const double *__restrict__ C,
                                                      double *__restrict__ M) {
  extern __shared__ double2 psm[];
  const int tid = threadIdx.x, e = blockIdx.x * blockDim.x + tid;
  const int w = blockIdx.y, r = blockIdx.z;
  for (int i = tid; i < Lq * ny; i += blockDim.x) psm[i] = ((const double2 *)phy)[i];
  __syncthreads();
  if (e >= BB) return;
  const double *X = ((w == 0) ? P : C) + 2 * ((size_t)(x0 + r) * Lq * BB + e);
  double ar[NYMAX], ai[NYMAX];
#pragma unroll
  for (int y = 0; y < NYMAX; ++y) ar[y] = ai[y] = 0.0;
#pragma unroll 8
  for (int qy = 0; qy < Lq; ++qy) {
    const double2 x = *(const double2 *)(X + 2 * (size_t)qy * BB);
#pragma unroll
    for (int y = 0; y < NYMAX; ++y)
      if (y < ny) {
        const double2 p = psm[qy * ny + y];
        ar[y] = fma(p.x, x.x, fma(-p.y, x.y, ar[y]));
        ai[y] = fma(p.x, x.y, fma(p.y, x.x, ai[y]));
      }
  }
  double *o = M + 2 * (((size_t)r * 2 + w) * ny * BB + e);
#pragma unroll
  for (int y = 0; y < NYMAX; ++y)
    if (y < ny) *(double2 *)(o + 2 * (size_t)y * BB) = make_double2(ar[y], ai[y]);
}

// real[w][iD][e] (+)= sum_{r < nr} e^{2 pi i (x0 + r) rho_x / Lq} M[r][w][s(iD)][e]:
// one thread per (e, slot s, w) reads its row sums once and updates the (at
// most nine) rho of the slot, dslot[s][j] = iD | (rho_x mod Lq) << 16 or -1;
// the first pass writes, the last one scales by 1/Nq
__global__ __launch_bounds__(256) void ft_cols_kernel(int BB, int Lq, int nD, int ny, int x0, int nr, int first,
                                                      double scale, const double *__restrict__ twq,
                                                      const int *__restrict__ dslot, const double *__restrict__ M,
                                                      double *__restrict__ real) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = blockIdx.y, w = blockIdx.z;
  if (e >= BB) return;
  int ent[NYMAX];
  double sr[NYMAX], si[NYMAX];
#pragma unroll
  for (int j = 0; j < NYMAX; ++j) {
    ent[j] = dslot[sl * NYMAX + j];
    sr[j] = si[j] = 0.0;
    if (ent[j] >= 0 && !first) {
      const size_t o = ((size_t)w * nD + (ent[j] & 0xffff)) * BB + e;
      sr[j] = real[2 * o];
      si[j] = real[2 * o + 1];
    }
  }
  for (int r = 0; r < nr; ++r) {
    const double2 a = *(const double2 *)(M + 2 * ((((size_t)r * 2 + w) * ny + sl) * BB + e));
#pragma unroll
    for (int j = 0; j < NYMAX; ++j)
      if (ent[j] >= 0) {
        const double2 tw = ((const double2 *)twq)[((x0 + r) * (ent[j] >> 16)) % Lq];
        sr[j] = fma(tw.x, a.x, fma(-tw.y, a.y, sr[j]));
        si[j] = fma(tw.x, a.y, fma(tw.y, a.x, si[j]));
      }
  }
#pragma unroll
  for (int j = 0; j < NYMAX; ++j)
    if (ent[j] >= 0) {
      const size_t o = ((size_t)w * nD + (ent[j] & 0xffff)) * BB + e;
      real[2 * o] = sr[j] * scale;
      real[2 * o + 1] = si[j] * scale;
    }
}

size_t proj_ws_row_doubles(const ProjArgs &a) { return 2 * 2 * (size_t)a.ny * a.B * a.B; }

static int proj_rows_per_pass(const ProjArgs &a, size_t ws_doubles, int rmax) {
  const size_t per_row = 2 * 2 * (size_t)a.ny * a.B * a.B;  // doubles of M per qx row
  return (int)std::max<size_t>(1, std::min<size_t>({(size_t)a.Lq, (size_t)rmax, ws_doubles / per_row}));
}

hipError_t launch_ft(const ProjArgs &a, const double *P, const double *C, double *ws, size_t ws_doubles,
                     double *real, hipStream_t st) {
  const int BB = a.B * a.B;
  if (a.ny < 1 || a.ny > NYMAX || a.Nq != a.Lq * a.Lq || a.nD > 65535) return hipErrorInvalidValue;
  const size_t per_row = 2 * 2 * (size_t)a.ny * BB;
  if (ws_doubles < per_row) return hipErrorInvalidValue;
  const int R = proj_rows_per_pass(a, ws_doubles, a.Lq);
  const size_t lds = sizeof(double2) * (size_t)a.Lq * a.ny;
  for (int x0 = 0; x0 < a.Lq; x0 += R) {
    const int nr = std::min(R, a.Lq - x0);
    hipLaunchKernelGGL(ft_rows_kernel, dim3((BB + 255) / 256, 2, nr), dim3(256), lds, st, BB, a.Lq, a.ny, x0, a.phy,
                       P, C, ws);
    hipLaunchKernelGGL(ft_cols_kernel, dim3((BB + 255) / 256, a.ny, 2), dim3(256), 0, st, BB, a.Lq, a.nD, a.ny, x0,
                       nr, x0 == 0 ? 1 : 0, x0 + nr >= a.Lq ? 1.0 / (double)a.Nq : 1.0, a.twq, a.dslot, ws, real);
  }
  return hipGetLastError();
}

// G[w][iD][row][col]; w = 0 feeds VP (from C), w = 1 feeds VC (from P and C)
__global__ void gather_kernel(int n_o, int n_ff, int B, int nD, const int *__restrict__ ff,
                              const int *__restrict__ dlist, const int *__restrict__ ffgrid,
                              const int *__restrict__ dgrid, const double *__restrict__ real,
                              double *__restrict__ G) {
  const long long BB = (long long)B * B;
  const long long total = 2LL * nD * BB;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int col = (int)(i % B), row = (int)((i / B) % B);
  const int iD = (int)((i / BB) % nD);
  const int w = (int)(i / (BB * nD));
  const int no2 = n_o * n_o;
  const int r = row / no2, a = (row % no2) / n_o, b = row % n_o;
  const int rp = col / no2, c = (col % no2) / n_o, d = col % n_o;
  const int Rx = ff[2 * r], Ry = ff[2 * r + 1], Rpx = ff[2 * rp], Rpy = ff[2 * rp + 1];
  const int px = dlist[2 * iD], py = dlist[2 * iD + 1];
  auto fidx = [&](int x, int y) -> int {
    if (x < -8 || x > 8 || y < -8 || y > 8) return -1;
    return ffgrid[(x + 8) * 17 + (y + 8)];
  };
  auto didx = [&](int x, int y) -> int {
    if (x < -8 || x > 8 || y < -8 || y > 8) return -1;
    return dgrid[(x + 8) * 17 + (y + 8)];
  };
  const double *Pr = real;               // P(rho) at w = 0 slot
  const double *Cr = real + 2 * nD * BB;  // C(rho) at w = 1 slot
  double gr = 0.0, gi = 0.0;
  const int A = fidx(Rx + px, Ry + py), Bi = fidx(Rpx - px, Rpy - py);
  if (w == 0) {
    if (A >= 0 && Bi >= 0) {
      const size_t s = (size_t)iD * BB + (size_t)(A * no2 + a * n_o + d) * B + (Bi * no2 + c * n_o + b);
      gr += Cr[2 * s];
      gi += Cr[2 * s + 1];
    }
    const int A2 = fidx(Rx + px - Rpx, Ry + py - Rpy), B2 = fidx(-px, -py);
    const int D2 = didx(px - Rpx, py - Rpy);
    if (A2 >= 0 && B2 >= 0 && D2 >= 0) {
      const size_t s = (size_t)D2 * BB + (size_t)(A2 * no2 + a * n_o + c) * B + (B2 * no2 + d * n_o + b);
      gr -= Cr[2 * s];
      gi -= Cr[2 * s + 1];
    }
  } else {
    if (A >= 0 && Bi >= 0) {
      const size_t s = (size_t)iD * BB + (size_t)(A * no2 + a * n_o + d) * B + (Bi * no2 + c * n_o + b);
      gr += Pr[2 * s];
      gi += Pr[2 * s + 1];
    }
    const int B4 = fidx(px, py), A4 = fidx(Rx - Rpx + px, Ry - Rpy + py);
    const int D4 = didx(-Rpx, -Rpy);
    if (A4 >= 0 && B4 >= 0 && D4 >= 0) {
      const size_t s = (size_t)D4 * BB + (size_t)(A4 * no2 + a * n_o + c) * B + (B4 * no2 + b * n_o + d);
      gr -= Cr[2 * s];
      gi -= Cr[2 * s + 1];
    }
  }
  G[2 * i] = gr;
  G[2 * i + 1] = gi;
}

// D[q][(R,a,b)][(R',c,d)] = -C[q][(R,a,c)][(R',b,d)]: the third channel in the
// layout of C, D_{n1n2n3n4} = -C_{n1n2n4n3}; a pure gather, exact
__global__ void channel_d_kernel(int n_o, int B, long long n, const double2 *__restrict__ C,
                                 double2 *__restrict__ D) {
  const int no2 = n_o * n_o;
  const long long BB = (long long)B * B;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(i % B), row = (int)((i / B) % B);
    const long long q = i / BB;
    const int r = row / no2, a = (row % no2) / n_o, b = row % n_o;
    const int rp = col / no2, c = (col % no2) / n_o, d = col % n_o;
    const double2 v = C[q * BB + (long long)(r * no2 + a * n_o + c) * B + (rp * no2 + b * n_o + d)];
    D[i] = make_double2(-v.x, -v.y);
  }
}

hipError_t launch_channel_d(int n_o, int B, int Nq, const double *C, double *D, hipStream_t st) {
  const long long n = (long long)Nq * B * B;
  const long long blocks = std::min<long long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(channel_d_kernel, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(256), 0, st, n_o, B, n,
                     (const double2 *)C, (double2 *)D);
  return hipGetLastError();
}

hipError_t launch_gather(const ProjArgs &a, const double *real, double *G, hipStream_t st) {
  const long long total = 2LL * a.nD * a.B * a.B;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a.n_o, a.n_ff, a.B,
                     a.nD, a.ff, a.dlist, a.ffgrid, a.dgrid, real, G);
  return hipGetLastError();
}

// M[r][w][s][e] = sum_{rho with s(rho) = s} e^{2 pi i (x0 + r) rho_x / Lq} G[w][rho][e]
// for r < nr; one thread per (e, s, w) keeps the nr row sums
__global__ __launch_bounds__(256) void assemble_rows_kernel(int BB, int Lq, int nD, int ny, int x0, int nr,
                                                            const double *__restrict__ twq,
                                                            const int *__restrict__ dtab,
                                                            const double *__restrict__ G, double *__restrict__ M) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = blockIdx.y, w = blockIdx.z;
  if (e >= BB) return;
  double hr[RMAX], hi[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) hr[r] = hi[r] = 0.0;
  for (int iD = 0; iD < nD; ++iD) {
    const int t = dtab[iD];
    if ((t >> 16) != sl) continue;  // uniform
    const int xv = t & 0xffff;
    const double2 g = *(const double2 *)(G + 2 * (((size_t)w * nD + iD) * BB + e));
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
      if (r < nr) {
        const double2 tw = ((const double2 *)twq)[((x0 + r) * xv) % Lq];
        hr[r] = fma(tw.x, g.x, fma(-tw.y, g.y, hr[r]));
        hi[r] = fma(tw.x, g.y, fma(tw.y, g.x, hi[r]));
      }
  }
#pragma unroll
  for (int r = 0; r < RMAX; ++r)
    if (r < nr) *(double2 *)(M + 2 * ((((size_t)r * 2 + w) * ny + sl) * BB + e)) = make_double2(hr[r], hi[r]);
}

// VX(x0 + r, qy)[e] = X[e] + X[V0][e] + sum_s e^{2 pi i qy y_s / Lq} M[r][w][s][e]
__global__ __launch_bounds__(256) void assemble_cols_kernel(int BB, int Lq, int ny, int x0,
                                                            const double *__restrict__ phy,
                                                            const double *__restrict__ P, const double *__restrict__ C,
                                                            const double *__restrict__ M,
                                                            const double *__restrict__ v0p,
                                                            const double *__restrict__ v0c, double *__restrict__ VP,
                                                            double *__restrict__ VC) {
  extern __shared__ double2 psm[];
  const int tid = threadIdx.x, e = blockIdx.x * blockDim.x + tid;
  const int w = blockIdx.y, r = blockIdx.z;
  for (int i = tid; i < Lq * ny; i += blockDim.x) psm[i] = ((const double2 *)phy)[i];
  __syncthreads();
  if (e >= BB) return;
  const double *v0 = (w == 0) ? v0p : v0c;
  const double v0r = v0[2 * e], v0i = v0[2 * e + 1];
  double hr[NYMAX], hi[NYMAX];
#pragma unroll
  for (int y = 0; y < NYMAX; ++y) {
    hr[y] = hi[y] = 0.0;
    if (y < ny) {
      const double2 h = *(const double2 *)(M + 2 * ((((size_t)r * 2 + w) * ny + y) * BB + e));
      hr[y] = h.x;
      hi[y] = h.y;
    }
  }
  const size_t row = (size_t)(x0 + r) * Lq * BB + e;
  const double *X = (w == 0) ? P : C;
  double *out = (w == 0) ? VP : VC;
#pragma unroll 8
  for (int qy = 0; qy < Lq; ++qy) {
    const double2 x = *(const double2 *)(X + 2 * (row + (size_t)qy * BB));
    double sr = x.x + v0r, si = x.y + v0i;
#pragma unroll
    for (int y = 0; y < NYMAX; ++y)
      if (y < ny) {
        const double2 p = psm[qy * ny + y];
        sr = fma(p.x, hr[y], fma(-p.y, hi[y], sr));
        si = fma(p.x, hi[y], fma(p.y, hr[y], si));
      }
    *(double2 *)(out + 2 * (row + (size_t)qy * BB)) = make_double2(sr, si);
  }
}

hipError_t launch_assemble(const ProjArgs &a, const double *P, const double *C, const double *G,
                           const double *v0p, const double *v0c, double *VP, double *VC, double *ws,
                           size_t ws_doubles, hipStream_t st, int nw) {
  const int BB = a.B * a.B;
  if (a.ny < 1 || a.ny > NYMAX || a.Nq != a.Lq * a.Lq || nw < 1 || nw > 2) return hipErrorInvalidValue;
  if (ws_doubles < 2 * 2 * (size_t)a.ny * BB) return hipErrorInvalidValue;
  const int R = proj_rows_per_pass(a, ws_doubles, RMAX);
  const size_t lds = sizeof(double2) * (size_t)a.Lq * a.ny;
  for (int x0 = 0; x0 < a.Lq; x0 += R) {
    const int nr = std::min(R, a.Lq - x0);
    hipLaunchKernelGGL(assemble_rows_kernel, dim3((BB + 255) / 256, a.ny, nw), dim3(256), 0, st, BB, a.Lq, a.nD,
                       a.ny, x0, nr, a.twq, a.dtab, G, ws);
    hipLaunchKernelGGL(assemble_cols_kernel, dim3((BB + 255) / 256, nw, nr), dim3(256), lds, st, BB, a.Lq, a.ny, x0,
                       a.phy, P, C, ws, v0p, v0c, VP, VC);
  }
  return hipGetLastError();
}

}  // namespace tufrg

// Orbital <-> band basis change of the exchange propagators (Sec. 4.1).
//
// The form-factor averages of the basis change,
//   U^{RR'}_{s1 s2 n1 n2}(s) = 1/N_f sum_k f_R(k) f*_R'(k) U_{s1 n1}(s - k) U_{s2 n2}(k)
//   X^{RR'}_{s1 s2 n1 n2}(u) = 1/N_f sum_k f_R(k) f*_R'(k) U_{s1 n1}(k) U*_{s2 n2}(k - u)
// (U(k): orbital rows, band columns; f_R(k) = e^{-ik.R}), depend on R and R'
// only through dR = R - R'.  In the bundle layout of the library (rows
// (R, a, b), columns (R', c, d)) the laws for P and C are plain sandwiches
// Pb = M^H P M, Cb = M^H C M (and the converses P = M Pb M^H, C = M Cb M^H) with
//   M_pp[(R,a,b),(R',c,d)] = U^{RR'}_{b a d c}(s) = 1/N_f sum_k e^{-ik.dR} U_ac(k) U_bd(s - k)
//   M_ph[(R,a,b),(R',c,d)] = X^{RR'}_{a b c d}(u) = 1/N_f sum_k e^{-ik.dR} U_ac(k) conj(U_bd(k - u)).
// basis_rows_kernel and basis_cols_kernel write the compact form
// Mc(q)[dR][(a, b, c, d)] (every dR of D = S - S); it is expanded to B x B like
// the loops, and zgemm_batched_kernel does the sandwich.
#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {
constexpr int ZT = 16;  // tile edge of the batched complex product
}  // namespace

// The phase is separable, e^{-ik.dR} = e^{-i kx dx} e^{-i ky dy}, so the k-sum
// runs in two passes over a chunk of coarse q:
//  rows: A[q][kx][y][(a,b,c,d)] = sum_ky e^{-i ky dy} U_ac(k) G_bd(k'), y = dy + NX;
//        one thread per (q, kx, y, a, b, c) streams the kx row (contiguous in
//        ky, the partner row backwards or forwards) and keeps the n_o values of d;
//  cols: Mc[q][dR][e] = 1/N_f sum_kx e^{-i kx dx} A[q][kx][dy + NX][e]; one
//        thread per (q, dR, e), consecutive e reading consecutive A.
// Every sum runs in a fixed order (deterministic).  CH = 0: pp (k' = s - k,
// G = U), 1: ph (k' = k - u, G = conj(U)).
template <int CH, int NX, int NO>
__global__ __launch_bounds__(256) void basis_rows_kernel(int Lq, int n_ref, int Lf, int q0, long long n_items,
                                                         const double2 *__restrict__ U,
                                                         const double2 *__restrict__ tw, double2 *__restrict__ A) {
  constexpr int NW = 2 * NX + 1, NO2 = NO * NO, NO3 = NO2 * NO, NO4 = NO2 * NO2;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_items) return;  // no barrier in this kernel
  const int abc = (int)(gid % NO3);
  const int y = (int)((gid / NO3) % NW);
  const long long row = gid / ((long long)NO3 * NW);  // qq * Lf + kx
  const int kx = (int)(row % Lf), qq = (int)(row / Lf);
  const int a = abc / NO2, b = (abc / NO) % NO, c = abc % NO;
  const int q = q0 + qq;
  const int qfx = (q / Lq) * n_ref, qfy = (q % Lq) * n_ref;
  int kpx = CH == 0 ? qfx - kx : kx - qfx;
  kpx = kpx < 0 ? kpx + Lf : kpx;
  const int dy = y - NX, sdy = dy < 0 ? dy + Lf : dy;
  const double2 *Uk = U + (size_t)kx * Lf * NO2 + a * NO + c;  // U_ac(kx, ky) at ky = 0
  const double2 *Up = U + (size_t)kpx * Lf * NO2 + b * NO;     // U_b.(k') row
  double sr[NO], si[NO];
#pragma unroll
  for (int d = 0; d < NO; ++d) sr[d] = si[d] = 0.0;
  int j = 0, kpy = CH == 0 ? qfy : (Lf - qfy) % Lf;  // partner y at ky = 0
  for (int ky = 0; ky < Lf; ++ky) {
    const double2 u = Uk[(size_t)ky * NO2];
    const double2 w = tw[j];  // e^{-i 2 pi ky dy / L_f}
    // w u, then times G_bd(k') for every d
    const double wr = w.x * u.x - w.y * u.y, wi = w.x * u.y + w.y * u.x;
    const double2 *v = Up + (size_t)kpy * NO2;
#pragma unroll
    for (int d = 0; d < NO; ++d) {
      const double2 g = v[d];
      const double gi = CH == 0 ? g.y : -g.y;
      sr[d] = fma(wr, g.x, fma(-wi, gi, sr[d]));
      si[d] = fma(wr, gi, fma(wi, g.x, si[d]));
    }
    j += sdy;
    j = j >= Lf ? j - Lf : j;
    if (CH == 0) {
      kpy = kpy == 0 ? Lf - 1 : kpy - 1;
    } else {
      kpy = kpy == Lf - 1 ? 0 : kpy + 1;
    }
  }
  double2 *dst = A + ((size_t)row * NW + y) * NO4 + ((a * NO + b) * NO + c) * NO;
#pragma unroll
  for (int d = 0; d < NO; ++d) dst[d] = make_double2(sr[d], si[d]);
}

// Two orbitals: one thread per (q, kx, a, b, c) does every dy of the box, so
// the loads of U_ac(k) and U_b.(k') serve 2 NX + 1 phases; the phase of dy
// is the dy-th power of e^{-i 2 pi ky / L_f} (one table load per k).
template <int CH, int NX>
__global__ __launch_bounds__(256) void basis_rows2_kernel(int Lq, int n_ref, int Lf, int q0, long long n_items,
                                                          const double2 *__restrict__ U,
                                                          const double2 *__restrict__ tw, double2 *__restrict__ A) {
  constexpr int NO = 2, NW = 2 * NX + 1, NO2 = 4, NO3 = 8, NO4 = 16;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_items) return;  // no barrier in this kernel
  const int abc = (int)(gid % NO3);
  const long long row = gid / NO3;  // qq * Lf + kx
  const int kx = (int)(row % Lf), qq = (int)(row / Lf);
  const int a = abc / NO2, b = (abc / NO) % NO, c = abc % NO;
  const int q = q0 + qq;
  const int qfx = (q / Lq) * n_ref, qfy = (q % Lq) * n_ref;
  int kpx = CH == 0 ? qfx - kx : kx - qfx;
  kpx = kpx < 0 ? kpx + Lf : kpx;
  const double2 *Uk = U + (size_t)kx * Lf * NO2 + a * NO + c;
  const double2 *Up = U + (size_t)kpx * Lf * NO2 + b * NO;
  double sr[NW][NO], si[NW][NO];
#pragma unroll
  for (int y = 0; y < NW; ++y)
#pragma unroll
    for (int d = 0; d < NO; ++d) sr[y][d] = si[y][d] = 0.0;
  int kpy = CH == 0 ? qfy : (Lf - qfy) % Lf;
  for (int ky = 0; ky < Lf; ++ky) {
    const double2 u = Uk[(size_t)ky * NO2];
    const double2 *v = Up + (size_t)kpy * NO2;
    double pr[NO], pi[NO];
#pragma unroll
    for (int d = 0; d < NO; ++d) {
      const double2 g = v[d];
      const double gi = CH == 0 ? g.y : -g.y;
      pr[d] = u.x * g.x - u.y * gi;
      pi[d] = u.x * gi + u.y * g.x;
    }
    // phases w^dy, dy = 1..NX, w = e^{-i 2 pi ky / L_f}; dy < 0 by conjugation
    double wr[NX + 1], wi[NX + 1];
    wr[0] = 1.0;
    wi[0] = 0.0;
    const double2 w1 = tw[ky];
    wr[1] = w1.x;
    wi[1] = w1.y;
#pragma unroll
    for (int m = 2; m <= NX; ++m) {
      wr[m] = wr[m - 1] * w1.x - wi[m - 1] * w1.y;
      wi[m] = wr[m - 1] * w1.y + wi[m - 1] * w1.x;
    }
#pragma unroll
    for (int y = 0; y < NW; ++y) {
      const int m = y < NX ? NX - y : y - NX;
      const double xr = wr[m], xi = y < NX ? -wi[m] : wi[m];
#pragma unroll
      for (int d = 0; d < NO; ++d) {
        sr[y][d] = fma(xr, pr[d], fma(-xi, pi[d], sr[y][d]));
        si[y][d] = fma(xr, pi[d], fma(xi, pr[d], si[y][d]));
      }
    }
    if (CH == 0) {
      kpy = kpy == 0 ? Lf - 1 : kpy - 1;
    } else {
      kpy = kpy == Lf - 1 ? 0 : kpy + 1;
    }
  }
#pragma unroll
  for (int y = 0; y < NW; ++y) {
    double2 *dst = A + ((size_t)row * NW + y) * NO4 + ((a * NO + b) * NO + c) * NO;
#pragma unroll
    for (int d = 0; d < NO; ++d) dst[d] = make_double2(sr[y][d], si[y][d]);
  }
}

__global__ __launch_bounds__(256) void basis_cols_kernel(int no4, int Lf, int NX, int q0, int nq, int nD,
                                                         const int *__restrict__ dlist,
                                                         const double2 *__restrict__ tw,
                                                         const double2 *__restrict__ A, double inv_nf,
                                                         double2 *__restrict__ out) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)nq * nD * no4) return;
  const int e = (int)(gid % no4), iD = (int)((gid / no4) % nD), qq = (int)(gid / ((long long)no4 * nD));
  const int NW = 2 * NX + 1, y = dlist[2 * iD + 1] + NX;
  const int dx = dlist[2 * iD], sdx = dx < 0 ? dx + Lf : dx;
  const double2 *src = A + ((size_t)qq * Lf * NW + y) * no4 + e;
  double sr = 0.0, si = 0.0;
  int j = 0;
  for (int kx = 0; kx < Lf; ++kx) {
    const double2 v = src[(size_t)kx * NW * no4];
    const double2 w = tw[j];  // e^{-i 2 pi kx dx / L_f}
    sr = fma(w.x, v.x, fma(-w.y, v.y, sr));
    si = fma(w.x, v.y, fma(w.y, v.x, si));
    j += sdx;
    j = j >= Lf ? j - Lf : j;
  }
  out[((size_t)(q0 + qq) * nD + iD) * no4 + e] = make_double2(sr * inv_nf, si * inv_nf);
}

size_t basis_rows_doubles(int n_o, int Lf, int box, int nq) {
  return 2 * (size_t)nq * Lf * (2 * box + 1) * n_o * n_o * n_o * n_o;
}

hipError_t launch_basis_compact(int channel, int n_o, int Lq, int n_ref, int nD, int box, const int *dlist,
                                const double *U, const double *tw, double *rows, int q_chunk, double *out,
                                hipStream_t st) {
  if ((channel != 0 && channel != 1) || (box != 2 && box != 4) || (n_o != 2 && n_o != 6) || q_chunk < 1)
    return hipErrorInvalidValue;
  const int Lf = Lq * n_ref, Nq = Lq * Lq, no4 = n_o * n_o * n_o * n_o;
  const int NW = 2 * box + 1;
  const double inv = 1.0 / ((double)Lf * Lf);
  const double2 *u = (const double2 *)U, *w = (const double2 *)tw;
  double2 *A = (double2 *)rows;
  for (int q0 = 0; q0 < Nq; q0 += q_chunk) {
    const int nq = Nq - q0 < q_chunk ? Nq - q0 : q_chunk;
    // two orbitals: a thread per (q, kx, a, b, c) for all dy; six: per (q, kx, dy, a, b, c)
    const long long n_items = (long long)nq * Lf * (n_o == 2 ? 1 : NW) * n_o * n_o * n_o;
    const dim3 grid1((unsigned)((n_items + 255) / 256)), block(256);
#define TUFRG_BASIS_ROWS(CH, NX, NO)                                                                                \
  hipLaunchKernelGGL((basis_rows_kernel<CH, NX, NO>), grid1, block, 0, st, Lq, n_ref, Lf, q0, n_items, u, w, A)
#define TUFRG_BASIS_ROWS2(CH, NX)                                                                                   \
  hipLaunchKernelGGL((basis_rows2_kernel<CH, NX>), grid1, block, 0, st, Lq, n_ref, Lf, q0, n_items, u, w, A)
    const int sel = channel * 4 + (box == 4 ? 2 : 0) + (n_o == 6 ? 1 : 0);
    switch (sel) {
      case 0: TUFRG_BASIS_ROWS2(0, 2); break;
      case 1: TUFRG_BASIS_ROWS(0, 2, 6); break;
      case 2: TUFRG_BASIS_ROWS2(0, 4); break;
      case 3: TUFRG_BASIS_ROWS(0, 4, 6); break;
      case 4: TUFRG_BASIS_ROWS2(1, 2); break;
      case 5: TUFRG_BASIS_ROWS(1, 2, 6); break;
      case 6: TUFRG_BASIS_ROWS2(1, 4); break;
      default: TUFRG_BASIS_ROWS(1, 4, 6); break;
    }
#undef TUFRG_BASIS_ROWS
#undef TUFRG_BASIS_ROWS2
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long n_out = (long long)nq * nD * no4;
    hipLaunchKernelGGL(basis_cols_kernel, dim3((unsigned)((n_out + 255) / 256)), block, 0, st, no4, Lf, box, q0, nq,
                       nD, dlist, w, (const double2 *)A, inv, (double2 *)out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Change of the form-factor basis: Y[q][(i,a,b),(j,c,d)] = sum_{R,R'} A_iR
// X[q][(R,a,b),(R',c,d)] conj(A_jR') (A = W for plane waves -> symmetrised
// form factors, A = W^H back); one thread per output entry, A in LDS.
__global__ __launch_bounds__(256) void ff_apply_kernel(int n_ff, int no2, int n_q, const double2 *__restrict__ A,
                                                       const double2 *__restrict__ X, double2 *__restrict__ Y) {
  __shared__ double2 sA[25 * 25];  // at most 25 form factors (|R_x|, |R_y| <= 2)
  for (int i = threadIdx.x; i < n_ff * n_ff; i += blockDim.x) sA[i] = A[i];
  __syncthreads();
  const int B = n_ff * no2;
  const long long BB = (long long)B * B;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)n_q * BB) return;
  const long long q = gid / BB;
  const int col = (int)(gid % B), row = (int)((gid / B) % B);
  const int i = row / no2, ab = row % no2, j = col / no2, cd = col % no2;
  const double2 *Xq = X + q * BB;
  double sr = 0.0, si = 0.0;
  for (int R = 0; R < n_ff; ++R) {
    const double2 a = sA[i * n_ff + R];
    if (a.x == 0.0 && a.y == 0.0) continue;
    double tr = 0.0, ti = 0.0;  // sum_R' X[(R,ab),(R',cd)] conj(A_jR')
    for (int Rp = 0; Rp < n_ff; ++Rp) {
      const double2 b = sA[j * n_ff + Rp];
      const double2 x = Xq[(long long)(R * no2 + ab) * B + Rp * no2 + cd];
      tr = fma(x.x, b.x, fma(x.y, b.y, tr));
      ti = fma(x.y, b.x, fma(-x.x, b.y, ti));
    }
    sr = fma(a.x, tr, fma(-a.y, ti, sr));
    si = fma(a.x, ti, fma(a.y, tr, si));
  }
  Y[gid] = make_double2(sr, si);
}

hipError_t launch_ff_apply(int n_ff, int no2, int n_q, const double *A, const double *X, double *Y, hipStream_t st) {
  if (n_ff < 1 || n_ff > 25 || no2 < 1 || n_q < 1) return hipErrorInvalidValue;
  const long long n = (long long)n_q * n_ff * no2 * n_ff * no2;
  hipLaunchKernelGGL(ff_apply_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n_ff, no2, n_q,
                     (const double2 *)A, (const double2 *)X, (double2 *)Y);
  return hipGetLastError();
}

// C[q] = opA(A[q]) opB(B[q]) for n x n complex matrices, op 0: as is, 1: conjugate transpose.
template <int TA, int TB>
__global__ __launch_bounds__(ZT *ZT) void zgemm_batched_kernel(int n, const double2 *__restrict__ A,
                                                               const double2 *__restrict__ Bm,
                                                               double2 *__restrict__ C) {
  __shared__ double2 sA[ZT][ZT + 1], sB[ZT][ZT + 1];
  const int tx = threadIdx.x % ZT, ty = threadIdx.x / ZT;
  const int i = blockIdx.y * ZT + ty, j = blockIdx.x * ZT + tx;
  const size_t base = (size_t)blockIdx.z * n * n;
  const double2 *Aq = A + base, *Bq = Bm + base;
  double cr = 0.0, ci = 0.0;
  for (int k0 = 0; k0 < n; k0 += ZT) {
    {
      const int r = i, col = k0 + tx;  // element (r, col) of opA(A)
      double2 v = make_double2(0.0, 0.0);
      if (r < n && col < n) {
        if (TA == 0) {
          v = Aq[(size_t)r * n + col];
        } else {
          v = Aq[(size_t)col * n + r];
          v.y = -v.y;
        }
      }
      sA[ty][tx] = v;
    }
    {
      const int r = k0 + ty, col = j;  // element (r, col) of opB(B)
      double2 v = make_double2(0.0, 0.0);
      if (r < n && col < n) {
        if (TB == 0) {
          v = Bq[(size_t)r * n + col];
        } else {
          v = Bq[(size_t)col * n + r];
          v.y = -v.y;
        }
      }
      sB[ty][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < ZT; ++kk) {
      const double2 x = sA[ty][kk], y = sB[kk][tx];
      cr = fma(x.x, y.x, fma(-x.y, y.y, cr));
      ci = fma(x.x, y.y, fma(x.y, y.x, ci));
    }
    __syncthreads();
  }
  if (i < n && j < n) C[base + (size_t)i * n + j] = make_double2(cr, ci);
}

hipError_t launch_zgemm_batched(int n, int n_q, int opA, int opB, const double *A, const double *Bm, double *C,
                                hipStream_t st) {
  if (n < 1 || n_q < 1 || !(opA == 0 || opB == 0) || opA < 0 || opA > 1 || opB < 0 || opB > 1)
    return hipErrorInvalidValue;
  const int tiles = (n + ZT - 1) / ZT;
  constexpr int QMAX = 65535;  // grid z limit: launch in slices of coarse q
  for (int q0 = 0; q0 < n_q; q0 += QMAX) {
    const int nq = n_q - q0 < QMAX ? n_q - q0 : QMAX;
    const size_t off = (size_t)q0 * n * n;
    const dim3 grid((unsigned)tiles, (unsigned)tiles, (unsigned)nq), block(ZT * ZT);
    const double2 *a = (const double2 *)A + off, *b = (const double2 *)Bm + off;
    double2 *c = (double2 *)C + off;
    if (opA == 0 && opB == 0)
      hipLaunchKernelGGL((zgemm_batched_kernel<0, 0>), grid, block, 0, st, n, a, b, c);
    else if (opA == 1)
      hipLaunchKernelGGL((zgemm_batched_kernel<1, 0>), grid, block, 0, st, n, a, b, c);
    else
      hipLaunchKernelGGL((zgemm_batched_kernel<0, 1>), grid, block, 0, st, n, a, b, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tufrg

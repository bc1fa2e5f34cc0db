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
// basis_compact_kernel writes the compact form Mc(q)[dR][(a, b, c, d)]; it is
// expanded to B x B like the loops, and zgemm_batched_kernel does the sandwich.
#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {
constexpr int BASIS_THREADS = 256;
constexpr int ZT = 16;  // tile edge of the batched complex product
}  // namespace

// One thread per (entry, dR) of one coarse q; a block holds epb entries of
// that q (epb * nD <= 256).  Every thread walks the whole fine mesh in a fixed
// order (deterministic), with the phase index (kx dx + ky dy) mod L_f and the
// partner point advanced incrementally.  CH = 0: pp (k' = s - k), 1: ph (k' = k - u).
template <int CH>
__global__ __launch_bounds__(BASIS_THREADS) void basis_compact_kernel(int n_o, int Lq, int n_ref, int Lf, int nD,
                                                                      int epb, const int *__restrict__ dlist,
                                                                      const double2 *__restrict__ U,
                                                                      const double2 *__restrict__ tw, double inv_nf,
                                                                      double2 *__restrict__ out) {
  const int no2 = n_o * n_o, no4 = no2 * no2;
  const int nchunk = (no4 + epb - 1) / epb;
  const int q = blockIdx.x / nchunk, chunk = blockIdx.x % nchunk;
  const int t = threadIdx.x;
  const int e = chunk * epb + t / nD, iD = t % nD;
  if (t >= epb * nD || e >= no4) return;  // no barrier in this kernel
  const int a = e / (n_o * no2), b = (e / no2) % n_o, c = (e / n_o) % n_o, d = e % n_o;
  const int sdx = ((dlist[2 * iD] % Lf) + Lf) % Lf, sdy = ((dlist[2 * iD + 1] % Lf) + Lf) % Lf;
  const int qfx = (q / Lq) * n_ref, qfy = (q % Lq) * n_ref;
  const int kpy0 = CH == 0 ? qfy : (Lf - qfy) % Lf;  // partner y at ky = 0
  double sr = 0.0, si = 0.0;
  int jrow = 0;  // kx dx mod L_f
  for (int kx = 0; kx < Lf; ++kx) {
    int kpx = CH == 0 ? qfx - kx : kx - qfx;
    kpx = kpx < 0 ? kpx + Lf : kpx;
    const double2 *Uk = U + (size_t)kx * Lf * no2 + a * n_o + c;   // U_ac(kx, ky) at ky = 0
    const double2 *Up = U + (size_t)kpx * Lf * no2 + b * n_o + d;  // U_bd(k') row
    int j = jrow, kpy = kpy0;
    for (int ky = 0; ky < Lf; ++ky) {
      const double2 u = Uk[(size_t)ky * no2];
      const double2 g = Up[(size_t)kpy * no2];
      const double gi = CH == 0 ? g.y : -g.y;
      const double pr = u.x * g.x - u.y * gi, pi = u.x * gi + u.y * g.x;
      const double2 w = tw[j];  // e^{-i 2 pi j / L_f}
      sr = fma(w.x, pr, fma(-w.y, pi, sr));
      si = fma(w.x, pi, fma(w.y, pr, si));
      j += sdy;
      j = j >= Lf ? j - Lf : j;
      if (CH == 0) {
        kpy = kpy == 0 ? Lf - 1 : kpy - 1;
      } else {
        kpy = kpy == Lf - 1 ? 0 : kpy + 1;
      }
    }
    jrow += sdx;
    jrow = jrow >= Lf ? jrow - Lf : jrow;
  }
  out[((size_t)q * nD + iD) * no4 + e] = make_double2(sr * inv_nf, si * inv_nf);
}

hipError_t launch_basis_compact(int channel, int n_o, int Lq, int n_ref, int nD, const int *dlist, const double *U,
                                const double *tw, double *out, hipStream_t st) {
  if (nD < 1 || nD > BASIS_THREADS || (channel != 0 && channel != 1)) return hipErrorInvalidValue;
  const int Lf = Lq * n_ref, no4 = n_o * n_o * n_o * n_o;
  const int epb = BASIS_THREADS / nD;
  const int nchunk = (no4 + epb - 1) / epb;
  const dim3 grid((unsigned)(Lq * Lq * nchunk)), block(BASIS_THREADS);
  const double inv = 1.0 / ((double)Lf * Lf);
  if (channel == 0)
    hipLaunchKernelGGL(basis_compact_kernel<0>, grid, block, 0, st, n_o, Lq, n_ref, Lf, nD, epb, dlist,
                       (const double2 *)U, (const double2 *)tw, inv, (double2 *)out);
  else
    hipLaunchKernelGGL(basis_compact_kernel<1>, grid, block, 0, st, n_o, Lq, n_ref, Lf, nD, epb, dlist,
                       (const double2 *)U, (const double2 *)tw, inv, (double2 *)out);
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

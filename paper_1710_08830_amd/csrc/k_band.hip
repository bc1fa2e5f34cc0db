// Band data on the refined k-mesh (setup, once per context).
//
// For every fine k = 2 pi (kx, ky) / Lf: H(k) = sum_R t(R) exp(i k.R), its
// eigenvalues E_m(k) and eigenvectors U(k) (the unitary of the paper's Sec. 4.1
// transformation between orbital and band basis), by cyclic complex Jacobi
// rotations in FP64, one thread per k.  The loops only need e_m = E_m - mu and
// the band projectors Pi_m(k)_{ac} = U_{am} conj(U_{cm}), which are stored
// Hermitian-packed: NO real diagonal entries, then (Re, Im) of every a < c.
#include "common.h"
#include "kernels.h"

namespace tufrg {

template <int NO>
__global__ __launch_bounds__(64) void band_kernel(int Lf, int n_hop, const int *__restrict__ hop_R,
                                                  const double *__restrict__ hop_t, double mu, int unit_pi,
                                                  double *__restrict__ e_out, double *__restrict__ pi_out,
                                                  float *__restrict__ e32, float *__restrict__ pi32) {
  const int Nf = Lf * Lf;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Nf) return;
  const int kx = k / Lf, ky = k - kx * Lf;
  double Ar[NO][NO], Ai[NO][NO], Vr[NO][NO], Vi[NO][NO];
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      Ar[i][j] = 0.0;
      Ai[i][j] = 0.0;
      Vr[i][j] = (i == j) ? 1.0 : 0.0;
      Vi[i][j] = 0.0;
    }
  for (int h = 0; h < n_hop; ++h) {
    long long ph = (long long)kx * hop_R[2 * h] + (long long)ky * hop_R[2 * h + 1];
    ph %= Lf;
    if (ph < 0) ph += Lf;
    double s, c;
    sincospi(2.0 * (double)ph / (double)Lf, &s, &c);
    const double *t = hop_t + (size_t)h * NO * NO * 2;
#pragma unroll
    for (int i = 0; i < NO; ++i)
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        double tr = t[2 * (i * NO + j)], ti = t[2 * (i * NO + j) + 1];
        Ar[i][j] += tr * c - ti * s;
        Ai[i][j] += tr * s + ti * c;
      }
  }
  // symmetrise exactly (Hermitian input up to rounding)
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    Ai[i][i] = 0.0;
#pragma unroll
    for (int j = i + 1; j < NO; ++j) {
      double r = 0.5 * (Ar[i][j] + Ar[j][i]), m = 0.5 * (Ai[i][j] - Ai[j][i]);
      Ar[i][j] = r;
      Ar[j][i] = r;
      Ai[i][j] = m;
      Ai[j][i] = -m;
    }
  }
  for (int sweep = 0; sweep < 12; ++sweep) {
    double off = 0.0, diag = 0.0;
#pragma unroll
    for (int i = 0; i < NO; ++i) {
      diag += Ar[i][i] * Ar[i][i];
#pragma unroll
      for (int j = i + 1; j < NO; ++j) off += Ar[i][j] * Ar[i][j] + Ai[i][j] * Ai[i][j];
    }
    if (off <= 1e-34 * (diag + 1e-300)) break;
#pragma unroll
    for (int p = 0; p < NO; ++p)
#pragma unroll
      for (int q = p + 1; q < NO; ++q) {
        const double gr = Ar[p][q], gi = Ai[p][q];
        const double r = sqrt(gr * gr + gi * gi);
        if (!(r > 1e-300)) continue;
        // phase: multiply column q by w = conj(g)/|g| (row q by conj(w)); A_pq becomes |g|
        const double wr = gr / r, wi = -gi / r;
#pragma unroll
        for (int i = 0; i < NO; ++i) {
          double xr = Ar[i][q], xi = Ai[i][q];
          Ar[i][q] = xr * wr - xi * wi;
          Ai[i][q] = xr * wi + xi * wr;
          xr = Vr[i][q];
          xi = Vi[i][q];
          Vr[i][q] = xr * wr - xi * wi;
          Vi[i][q] = xr * wi + xi * wr;
        }
#pragma unroll
        for (int j = 0; j < NO; ++j) {
          double xr = Ar[q][j], xi = Ai[q][j];
          Ar[q][j] = xr * wr + xi * wi;
          Ai[q][j] = -xr * wi + xi * wr;
        }
        Ar[p][q] = r;
        Ai[p][q] = 0.0;
        Ar[q][p] = r;
        Ai[q][p] = 0.0;
        Ai[q][q] = 0.0;
        // real rotation zeroing the (p, q) entry
        const double theta = (Ar[q][q] - Ar[p][p]) / (2.0 * r);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
        for (int i = 0; i < NO; ++i) {
          double ar = Ar[i][p], ai = Ai[i][p], br = Ar[i][q], bi = Ai[i][q];
          Ar[i][p] = c * ar - s * br;
          Ai[i][p] = c * ai - s * bi;
          Ar[i][q] = s * ar + c * br;
          Ai[i][q] = s * ai + c * bi;
          ar = Vr[i][p];
          ai = Vi[i][p];
          br = Vr[i][q];
          bi = Vi[i][q];
          Vr[i][p] = c * ar - s * br;
          Vi[i][p] = c * ai - s * bi;
          Vr[i][q] = s * ar + c * br;
          Vi[i][q] = s * ai + c * bi;
        }
#pragma unroll
        for (int j = 0; j < NO; ++j) {
          double ar = Ar[p][j], ai = Ai[p][j], br = Ar[q][j], bi = Ai[q][j];
          Ar[p][j] = c * ar - s * br;
          Ai[p][j] = c * ai - s * bi;
          Ar[q][j] = s * ar + c * br;
          Ai[q][j] = s * ai + c * bi;
        }
        Ar[p][q] = 0.0;
        Ai[p][q] = 0.0;
        Ar[q][p] = 0.0;
        Ai[q][p] = 0.0;
      }
  }
  // ascending order (selection sort with predicated column swaps)
  double ev[NO];
#pragma unroll
  for (int i = 0; i < NO; ++i) ev[i] = Ar[i][i];
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = i + 1; j < NO; ++j) {
      const bool sw = ev[j] < ev[i];
      double a = ev[i], b = ev[j];
      ev[i] = sw ? b : a;
      ev[j] = sw ? a : b;
#pragma unroll
      for (int r = 0; r < NO; ++r) {
        double xr = Vr[r][i], yr = Vr[r][j], xi = Vi[r][i], yi = Vi[r][j];
        Vr[r][i] = sw ? yr : xr;
        Vr[r][j] = sw ? xr : yr;
        Vi[r][i] = sw ? yi : xi;
        Vi[r][j] = sw ? xi : yi;
      }
    }
  const size_t Nfs = (size_t)Nf;
#pragma unroll
  for (int m = 0; m < NO; ++m) {
    const double e = ev[m] - mu;
    e_out[m * Nfs + k] = e;
    e32[m * Nfs + k] = (float)e;
    int comp = m * NO * NO;
    if (unit_pi) {
      // band basis: the single-particle basis is the eigenbasis, Pi_m = e_m e_m^T
#pragma unroll
      for (int i = 0; i < NO * NO; ++i) {
        const double v = (i < NO && i == m) ? 1.0 : 0.0;
        pi_out[(comp + i) * Nfs + k] = v;
        pi32[(comp + i) * Nfs + k] = (float)v;
      }
      continue;
    }
#pragma unroll
    for (int a = 0; a < NO; ++a) {
      double v = Vr[a][m] * Vr[a][m] + Vi[a][m] * Vi[a][m];
      pi_out[(comp + a) * Nfs + k] = v;
      pi32[(comp + a) * Nfs + k] = (float)v;
    }
    int off = comp + NO;
#pragma unroll
    for (int a = 0; a < NO; ++a)
#pragma unroll
      for (int c = a + 1; c < NO; ++c) {
        // U_am conj(U_cm)
        double re = Vr[a][m] * Vr[c][m] + Vi[a][m] * Vi[c][m];
        double im = Vi[a][m] * Vr[c][m] - Vr[a][m] * Vi[c][m];
        pi_out[off * Nfs + k] = re;
        pi_out[(off + 1) * Nfs + k] = im;
        pi32[off * Nfs + k] = (float)re;
        pi32[(off + 1) * Nfs + k] = (float)im;
        off += 2;
      }
  }
}

hipError_t launch_band(int n_o, int Lf, int n_hop, const int *hop_R, const double *hop_t, double mu, int unit_pi,
                       double *e, double *pi, float *e32, float *pi32, hipStream_t st) {
  const int Nf = Lf * Lf;
  dim3 grid((Nf + 63) / 64), block(64);
  switch (n_o) {
    case 1: hipLaunchKernelGGL(band_kernel<1>, grid, block, 0, st, Lf, n_hop, hop_R, hop_t, mu, unit_pi, e, pi, e32, pi32); break;
    case 2: hipLaunchKernelGGL(band_kernel<2>, grid, block, 0, st, Lf, n_hop, hop_R, hop_t, mu, unit_pi, e, pi, e32, pi32); break;
    case 4: hipLaunchKernelGGL(band_kernel<4>, grid, block, 0, st, Lf, n_hop, hop_R, hop_t, mu, unit_pi, e, pi, e32, pi32); break;
    case 6: hipLaunchKernelGGL(band_kernel<6>, grid, block, 0, st, Lf, n_hop, hop_R, hop_t, mu, unit_pi, e, pi, e32, pi32); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Regulator value per band and fine k at one scale: K (deriv) or J.  The
// input e is band-major [n_o][Nf]; the output is band-major too (aos_no = 0)
// or k-major [Nf][n_o] (aos_no = n_o).
__global__ void kval_kernel(int n, int Nf, int aos_no, const double *__restrict__ e, double lam, int scheme,
                            int deriv, double *__restrict__ kv, float *__restrict__ kv32) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = cut_val(e[i], lam, scheme, deriv);
  const int o = aos_no ? (i % Nf) * aos_no + i / Nf : i;
  kv[o] = v;
  kv32[o] = (float)v;
}

hipError_t launch_kval(int n, int Nf, int aos_no, const double *e, double lam, int scheme, int deriv, double *kv,
                       float *kv32, hipStream_t st) {
  hipLaunchKernelGGL(kval_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, Nf, aos_no, e, lam, scheme, deriv, kv,
                     kv32);
  return hipGetLastError();
}

// two orbitals, band layout [e_0][e_1][Pi_0 d0][Pi_0 d1][Pi_0 re][Pi_0 im]...:
// per k the 4-vector (e_0, e_1, K(e_0), K(e_1)) at scale lam
__global__ void ekv4_kernel(int Nf, const double *__restrict__ band, double lam, int scheme, int deriv,
                            double *__restrict__ ekv, float *__restrict__ ekv32) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Nf) return;
  const double e0 = band[k], e1 = band[(size_t)Nf + k];
  const double v[4] = {e0, e1, cut_val(e0, lam, scheme, deriv), cut_val(e1, lam, scheme, deriv)};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ekv[4 * (size_t)k + j] = v[j];
    ekv32[4 * (size_t)k + j] = (float)v[j];
  }
}

hipError_t launch_ekv4(int Nf, const double *band, double lam, int scheme, int deriv, double *ekv, float *ekv32,
                       hipStream_t st) {
  hipLaunchKernelGGL(ekv4_kernel, dim3((Nf + 255) / 256), dim3(256), 0, st, Nf, band, lam, scheme, deriv, ekv,
                     ekv32);
  return hipGetLastError();
}

// shell factors (a, b) of band m at k (see shell_ab)
__global__ void shell_ab_kernel(int n_o, int Nf, const double *__restrict__ e, double lam, int deriv,
                                double *__restrict__ cv, float *__restrict__ cv32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // i = m * Nf + k
  if (i >= n_o * Nf) return;
  const int m = i / Nf, k = i - m * Nf;
  double a, b;
  shell_ab(e[i], lam, deriv, a, b);
  const size_t ia = n_o == 2 ? 4 * (size_t)k + m : 2 * ((size_t)k * n_o + m);
  const size_t ib = n_o == 2 ? ia + 2 : ia + 1;
  cv[ia] = a;
  cv[ib] = b;
  cv32[ia] = (float)a;
  cv32[ib] = (float)b;
}

hipError_t launch_shell_ab(int n_o, int Nf, const double *e, double lam, int deriv, double *cv, float *cv32,
                           hipStream_t st) {
  const int n = n_o * Nf;
  hipLaunchKernelGGL(shell_ab_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n_o, Nf, e, lam, deriv, cv, cv32);
  return hipGetLastError();
}

// per k the 4-vector (Pi_0[00], Pi_0[11], Re Pi_0[01], Im Pi_0[01])
__global__ void pi4_kernel(int Nf, const double *__restrict__ band, double *__restrict__ pi4,
                           float *__restrict__ pi4_32) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Nf) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double v = band[(size_t)(2 + j) * Nf + k];
    pi4[4 * (size_t)k + j] = v;
    pi4_32[4 * (size_t)k + j] = (float)v;
  }
}

hipError_t launch_pi4(int Nf, const double *band, double *pi4, float *pi4_32, hipStream_t st) {
  hipLaunchKernelGGL(pi4_kernel, dim3((Nf + 255) / 256), dim3(256), 0, st, Nf, band, pi4, pi4_32);
  return hipGetLastError();
}

// component-major [nc][Nf] -> k-major [Nf][nc], FP64 and FP32 copies
__global__ void to_kmajor_kernel(int nc, int Nf, const double *__restrict__ src, double *__restrict__ dst,
                                 float *__restrict__ dst32) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nc * Nf) return;
  const int r = (int)(i % nc);
  const long long k = i / nc;
  const double v = src[(size_t)r * Nf + k];
  dst[i] = v;
  dst32[i] = (float)v;
}

hipError_t launch_to_kmajor(int nc, int Nf, const double *src, double *dst, float *dst32, hipStream_t st) {
  const long long n = (long long)nc * Nf;
  hipLaunchKernelGGL(to_kmajor_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nc, Nf, src, dst, dst32);
  return hipGetLastError();
}

}  // namespace tufrg

namespace tufrg {

// packed projectors -> Pi[m][k][a][c] (complex)
__global__ void unpack_pi_kernel(int n_o, int Nf, const double *__restrict__ pi, double *__restrict__ out) {
  const int no2 = n_o * n_o;
  const long long total = (long long)n_o * Nf * no2;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int c = (int)(i % n_o), a = (int)((i / n_o) % n_o);
  const long long k = (i / no2) % Nf;
  const int m = (int)(i / ((long long)no2 * Nf));
  const size_t base = (size_t)m * no2;
  double re, im = 0.0;
  if (a == c) {
    re = pi[(base + a) * Nf + k];
  } else {
    const int lo = a < c ? a : c, hi = a < c ? c : a;
    int p = 0;
    for (int x = 0; x < lo; ++x) p += n_o - 1 - x;
    p += hi - lo - 1;
    re = pi[(base + n_o + 2 * p) * Nf + k];
    im = pi[(base + n_o + 2 * p + 1) * Nf + k];
    if (a > c) im = -im;
  }
  out[2 * i] = re;
  out[2 * i + 1] = im;
}

hipError_t launch_unpack_pi(int n_o, int Nf, const double *pi, double *out, hipStream_t st) {
  const long long total = (long long)n_o * Nf * n_o * n_o;
  hipLaunchKernelGGL(unpack_pi_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n_o, Nf, pi, out);
  return hipGetLastError();
}

}  // namespace tufrg

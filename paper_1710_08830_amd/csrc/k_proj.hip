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
//   ft_kernel      X(q) -> X(rho)   (HBM read of both states)
//   gather_kernel  X(rho) -> G_P(rho), G_C(rho)
//   assemble       G(rho) -> VP(q), VC(q)  (HBM read of the states, write of V)
#include "common.h"
#include "kernels.h"

namespace tufrg {

// part[qc][w][iD][e] = sum_{q in chunk qc} e^{iq.rho_iD} X_w(q)[e]
// phq[q][iD] = e^{i q.rho_iD}: staged per tile of PQT q in LDS (every lane
// reads the same phase: broadcast)
constexpr int PQT = 16;
template <int NDP>
__global__ __launch_bounds__(256) void ft_kernel(int BB, int Nq, int nD, int qper, const double *__restrict__ phq,
                                                 const double *__restrict__ P, const double *__restrict__ C,
                                                 double *__restrict__ part) {
  __shared__ double2 sph[PQT][NDP];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y;
  const int qc = blockIdx.z;
  const bool active = e < BB;
  const double *X = (w == 0) ? P : C;
  double ar[NDP], ai[NDP];
#pragma unroll
  for (int i = 0; i < NDP; ++i) {
    ar[i] = 0.0;
    ai[i] = 0.0;
  }
  const int q0 = qc * qper, q1 = min(Nq, q0 + qper);
  for (int qb = q0; qb < q1; qb += PQT) {
    const int nqb = min(PQT, q1 - qb);
    __syncthreads();
    for (int i = threadIdx.x; i < nqb * nD; i += blockDim.x) {
      const int qq = i / nD, d = i - qq * nD;
      sph[qq][d] = *(const double2 *)(phq + 2 * ((size_t)(qb + qq) * nD + d));
    }
    __syncthreads();
    if (active) {
      for (int qq = 0; qq < nqb; ++qq) {
        const double2 x = *(const double2 *)(X + 2 * ((size_t)(qb + qq) * BB + e));
#pragma unroll
        for (int i = 0; i < NDP; ++i) {
          if (i < nD) {
            const double2 p = sph[qq][i];
            ar[i] = fma(p.x, x.x, fma(-p.y, x.y, ar[i]));
            ai[i] = fma(p.x, x.y, fma(p.y, x.x, ai[i]));
          }
        }
      }
    }
  }
  if (!active) return;
  const size_t base = ((size_t)qc * 2 + w) * nD;
#pragma unroll
  for (int i = 0; i < NDP; ++i)
    if (i < nD) {
      part[2 * ((base + i) * BB + e)] = ar[i];
      part[2 * ((base + i) * BB + e) + 1] = ai[i];
    }
}

__global__ void ft_reduce_kernel(long long n, int nqc, double scale, const double *__restrict__ part,
                                 double *__restrict__ real) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < nqc; ++c) s += part[(size_t)c * n + i];
  real[i] = s * scale;
}

hipError_t launch_ft(const ProjArgs &a, const double *P, const double *C, double *part, int nqc, double *real,
                     hipStream_t st) {
  const int BB = a.B * a.B;
  const int qper = (a.Nq + nqc - 1) / nqc;
  dim3 grid((BB + 255) / 256, 2, nqc), block(256);
  if (a.nD <= 13)
    hipLaunchKernelGGL(ft_kernel<13>, grid, block, 0, st, BB, a.Nq, a.nD, qper, a.phq, P, C, part);
  else if (a.nD <= 25)
    hipLaunchKernelGGL(ft_kernel<25>, grid, block, 0, st, BB, a.Nq, a.nD, qper, a.phq, P, C, part);
  else if (a.nD <= 41)
    hipLaunchKernelGGL(ft_kernel<41>, grid, block, 0, st, BB, a.Nq, a.nD, qper, a.phq, P, C, part);
  else
    return hipErrorInvalidValue;
  const long long n = 2LL * 2 * a.nD * BB;  // doubles per chunk
  hipLaunchKernelGGL(ft_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, nqc,
                     1.0 / (double)a.Nq, part, real);
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

hipError_t launch_gather(const ProjArgs &a, const double *real, double *G, hipStream_t st) {
  const long long total = 2LL * a.nD * a.B * a.B;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a.n_o, a.n_ff, a.B,
                     a.nD, a.ff, a.dlist, a.ffgrid, a.dgrid, real, G);
  return hipGetLastError();
}

// VX(q)[e] = X(q)[e] + X[V0][e] + sum_rho e^{iq.rho} G_X(rho)[e]; the phases of
// a tile of PQT q are staged in LDS as in ft_kernel
template <int NDP>
__global__ __launch_bounds__(256) void assemble_kernel(int BB, int Nq, int nD, int qper, const double *__restrict__ phq,
                                                       const double *__restrict__ P, const double *__restrict__ C,
                                                       const double *__restrict__ G, const double *__restrict__ v0p,
                                                       const double *__restrict__ v0c, double *__restrict__ VP,
                                                       double *__restrict__ VC) {
  __shared__ double2 sph[PQT][NDP];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y, qc = blockIdx.z;
  const bool active = e < BB;
  const int ea = active ? e : 0;
  const double *X = (w == 0) ? P : C;
  const double *v0 = (w == 0) ? v0p : v0c;
  double *out = (w == 0) ? VP : VC;
  double gr[NDP], gi[NDP];
#pragma unroll
  for (int i = 0; i < NDP; ++i) {
    if (i < nD) {
      const size_t s = ((size_t)w * nD + i) * BB + ea;
      gr[i] = G[2 * s];
      gi[i] = G[2 * s + 1];
    } else {
      gr[i] = 0.0;
      gi[i] = 0.0;
    }
  }
  const double v0r = v0[2 * ea], v0i = v0[2 * ea + 1];
  const int q0 = qc * qper, q1 = min(Nq, q0 + qper);
  for (int qb = q0; qb < q1; qb += PQT) {
    const int nqb = min(PQT, q1 - qb);
    __syncthreads();
    for (int i = threadIdx.x; i < nqb * nD; i += blockDim.x) {
      const int qq = i / nD, d = i - qq * nD;
      sph[qq][d] = *(const double2 *)(phq + 2 * ((size_t)(qb + qq) * nD + d));
    }
    __syncthreads();
    if (active) {
      for (int qq = 0; qq < nqb; ++qq) {
        const int q = qb + qq;
        const double2 x = *(const double2 *)(X + 2 * ((size_t)q * BB + e));
        double sr = x.x + v0r, si = x.y + v0i;
#pragma unroll
        for (int i = 0; i < NDP; ++i) {
          if (i < nD) {
            const double2 p = sph[qq][i];
            sr = fma(p.x, gr[i], fma(-p.y, gi[i], sr));
            si = fma(p.x, gi[i], fma(p.y, gr[i], si));
          }
        }
        double2 o;
        o.x = sr;
        o.y = si;
        *(double2 *)(out + 2 * ((size_t)q * BB + e)) = o;
      }
    }
  }
}

hipError_t launch_assemble(const ProjArgs &a, const double *P, const double *C, const double *G,
                           const double *v0p, const double *v0c, double *VP, double *VC, hipStream_t st) {
  const int BB = a.B * a.B;
  // enough q chunks to give every CU work
  int nqc = (int)((1024LL * 256 + 2LL * BB - 1) / (2LL * BB));
  nqc = max(1, min(nqc, a.Nq));
  const int qper = (a.Nq + nqc - 1) / nqc;
  nqc = (a.Nq + qper - 1) / qper;
  dim3 grid((BB + 255) / 256, 2, nqc), block(256);
  if (a.nD <= 13)
    hipLaunchKernelGGL(assemble_kernel<13>, grid, block, 0, st, BB, a.Nq, a.nD, qper, a.phq, P, C, G, v0p, v0c,
                       VP, VC);
  else if (a.nD <= 25)
    hipLaunchKernelGGL(assemble_kernel<25>, grid, block, 0, st, BB, a.Nq, a.nD, qper, a.phq, P, C, G, v0p, v0c,
                       VP, VC);
  else if (a.nD <= 41)
    hipLaunchKernelGGL(assemble_kernel<41>, grid, block, 0, st, BB, a.Nq, a.nD, qper, a.phq, P, C, G, v0p, v0c,
                       VP, VC);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace tufrg

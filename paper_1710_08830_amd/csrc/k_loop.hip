// Form-factor projected orbital loops (hot path).
//
// Loop matrices in the orbital basis (the paper's Sec. 3.1 loop matrices with
// the orbital-basis loop of Sec. 4.2, written as a direct k-sum on the refined
// mesh), in the bundle layout of the library:
//
//   Lpp(s)[(R1,a,b),(R2,c,d)] = 1/Nf sum_k e^{-ik.(R1-R2)}
//        sum_mn Pi_m(k)_ac Pi_n(s-k)_bd L-(e_m(k), e_n(s-k))
//   Lph(u)[(R1,a,b),(R2,c,d)] = 1/Nf sum_k e^{-ik.(R1-R2)}
//        sum_mn Pi_m(k)_ac Pi_n(k-u)_db L+(e_m(k), e_n(k-u))
//
// Both depend on R1, R2 only through dR = R1 - R2, so the kernel produces the
// compact loop  Lc(q)[dR][tau],  tau = (a, b, c, d) flattened.
//
// Two spin-orbitals (this kernel):
// * Completeness, Pi_1 = 1 - Pi_0, gives with X_n the projector at k' (its
//   transpose for ph) and alpha_m = L_m0 - L_m1:
//     W_m = sum_n L_mn X_n = alpha_m X_0 + L_m1 1,  M = sum_m Pi_m (x) W_m
//         = Pi_0 (x) (W_0 - W_1) + 1 (x) W_1,
//   so only e_0, e_1, K_0, K_1 and the four reals of Pi_0 are read per point,
//   as two 4-vectors (k-major arrays ekv and pi4).
// * M[(c,d,a,b)] = conj(M[(a,b,c,d)]): only 10 entries are distinct (4 real).
//   With the phase p = c + i s the accumulation of p M and p conj(M) needs only
//   A = sum c M and B = sum s M; the pair is rebuilt at the end as
//   A + iB and (A.re + B.im) + i (B.re - A.im).
// * The phase is separable, e^{-ik.dR} = e^{-i kx dx} e^{-i ky dy}: every lane
//   owns one ky and walks kx, so the kx phases are wave-uniform; accumulators
//   cover dx >= 0 only (dx < 0 follows from hermiticity,
//   Lc[dR][(ab,cd)] = conj(Lc[-dR][(cd,ab)])).  At the end of a kx chunk the
//   lanes' values are transposed through LDS and contracted with e^{-i ky dy}.
// Partial sums per (ky block, kx chunk) go to HBM in FP64; a finalising kernel
// adds them in a fixed order (deterministic, no atomics).
#include <vector>

#include "common.h"
#include "kernels.h"

namespace tufrg {

namespace {

// distinct entries: 4 real (tau = 0, 5, 10, 15) and 6 complex representatives
// (tau = 1, 11, 2, 7, 3, 6) with partners (4, 14, 8, 13, 12, 9)
constexpr int NREAL = 4, NCPLX = 6;
__device__ constexpr int REAL_TAU[NREAL] = {0, 5, 10, 15};
__device__ constexpr int CPLX_TAU[NCPLX] = {1, 11, 2, 7, 3, 6};
__device__ constexpr int CPLX_PARTNER[NCPLX] = {4, 14, 8, 13, 12, 9};

template <typename T, int SCHEME>
__device__ inline bool nondegenerate(T den, T x, T y, T lam) {
  if constexpr (dd_scheme(SCHEME) == CUT_TEMPERATURE)
    return fabs(den) > degen_rel<T>::v * lam;
  else
    return fabs(den) > degen_rel<T>::v * (lam + fabs(x) + fabs(y));
}

}  // namespace

template <typename T>
__device__ inline T ldb(const T *base, unsigned byte_off) {
  // base pointer is wave-uniform, the offset a 32-bit lane value
  return *(const T *)((const char *)base + byte_off);
}

// four consecutive values at index i of a k-major array of 4-vectors
template <typename T>
struct V4 {
  T x, y, z, w;
};
// Raw buffer loads: a descriptor of an array of nbytes bytes (base address,
// no stride, the gfx9-family data-format bits in the last word), a wave-uniform
// byte offset and a per-lane 32-bit byte offset.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
__device__ f32x4v raw_buffer_load_v4f32(i32x4 rsrc, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.raw.buffer.load.v4f32");
template <typename T>
__device__ inline i32x4 make_rsrc(const T *p, unsigned nbytes) {
  const unsigned long long a = (unsigned long long)p;
  return i32x4{(int)(unsigned)a, (int)(unsigned)(a >> 32), (int)nbytes, 0x00020000};
}
// four floats at byte offset soff (wave-uniform) + voff (per lane)
__device__ inline V4<float> ld4_buf(i32x4 r, unsigned voff, unsigned soff) {
  const f32x4v v = raw_buffer_load_v4f32(r, (int)voff, (int)soff, 0);
  return {v[0], v[1], v[2], v[3]};
}
// four doubles: two 16-byte loads
__device__ inline V4<double> ld4d_buf(i32x4 r, unsigned voff, unsigned soff) {
  const double2 a = __builtin_bit_cast(double2, raw_buffer_load_v4f32(r, (int)voff, (int)soff, 0));
  const double2 b = __builtin_bit_cast(double2, raw_buffer_load_v4f32(r, (int)voff + 16, (int)soff, 0));
  return {a.x, a.y, b.x, b.y};
}

// Loop body of one channel (CH = 0: pp, k' = q - k; CH = 1: ph, k' = k - q).
// ekv[k] = (e_0, e_1, K(e_0), K(e_1)), pi4[k] = (Pi_0[00], Pi_0[11], Re Pi_0[01], Im Pi_0[01]);
// shell scheme: K is the fixed-temperature J and cv[k] = (a_0, a_1, b_0, b_1)
// the shell factors; twk: exp(-2 pi i j / Lf) in the arithmetic type.
template <typename T, int NDX, int SCHEME, int CH>
__device__ inline void loop_no2_body(const T *__restrict__ ekv, const T *__restrict__ pi4,
                                     const T *__restrict__ cvp,
                                     const T *__restrict__ twk, int Lf, int qfx, int qfy, int ky, int x0,
                                     int x1, T lam, int deriv, T (&Sr)[NREAL], T (&Sc)[NCPLX][2],
                                     T (&Ar)[NDX - 1][NREAL], T (&Br)[NDX - 1][NREAL],
                                     T (&Ac)[NDX - 1][NCPLX][2], T (&Bc)[NDX - 1][NCPLX][2]) {
  constexpr T sg = (CH == 0) ? T(1) : T(-1);
  int kpy = (CH == 0) ? (qfy - ky) : (ky - qfy);
  kpy = ((kpy % Lf) + Lf) % Lf;
  int kpx = (CH == 0) ? (qfx - x0) : (x0 - qfx);
  kpx = ((kpx % Lf) + Lf) % Lf;
  // phase indices (kx (d + 1)) mod Lf, advanced with kx (wave-uniform)
  int jd[NDX - 1];
#pragma unroll
  for (int d = 0; d < NDX - 1; ++d) jd[d] = (int)(((long long)x0 * (d + 1)) % Lf);
  constexpr bool SHELL = SCHEME == CUT_SHELL;
  struct Pt {
    V4<T> ek, pk, cv;
  };
  // point (row, col) of a k-major array: row = kx (wave-uniform), col = ky (per lane):
  // raw buffer loads, descriptor and row offset in scalar registers, the lane's
  // 32-bit byte offset as the only vector operand
  const unsigned nbytes = (unsigned)Lf * Lf * 4u * (unsigned)sizeof(T);
  const auto rs_e = make_rsrc(ekv, nbytes), rs_p = make_rsrc(pi4, nbytes);
  const auto rs_c = make_rsrc(SHELL ? cvp : ekv, nbytes);
  auto load = [&](unsigned row, unsigned col, Pt &p) {
    if constexpr (sizeof(T) == 4) {
      const unsigned soff = row * (unsigned)Lf * 16u, voff = col * 16u;
      p.ek = ld4_buf(rs_e, voff, soff);
      p.pk = ld4_buf(rs_p, voff, soff);
      if constexpr (SHELL) p.cv = ld4_buf(rs_c, voff, soff);
    } else {
      const unsigned soff = row * (unsigned)Lf * 32u, voff = col * 32u;
      p.ek = ld4d_buf(rs_e, voff, soff);
      p.pk = ld4d_buf(rs_p, voff, soff);
      if constexpr (SHELL) p.cv = ld4d_buf(rs_c, voff, soff);
    }
  };
  // k' row of the next kx
  auto next_kpx = [&]() {
    kpx += (CH == 0) ? -1 : 1;
    kpx = kpx < 0 ? kpx + Lf : (kpx >= Lf ? kpx - Lf : kpx);
  };
  // arithmetic of one k-point (k data ck, k' data cp), in kx order
  auto point = [&](const Pt &ck, const Pt &cp) {
      const T ekm[2] = {ck.ek.x, ck.ek.y}, Kkm[2] = {ck.ek.z, ck.ek.w};
      const T P0 = ck.pk.x, P1 = ck.pk.y, Pr = ck.pk.z, Pi = ck.pk.w;
      const T epn[2] = {cp.ek.x, cp.ek.y}, Kpn[2] = {cp.ek.z, cp.ek.w};
      const T X0 = cp.pk.x, X1 = cp.pk.y, Xr = cp.pk.z, Xi = sg * cp.pk.w;
      // loop kernels L_mn: pp (K(e1)+K(e2))/(e1+e2), ph -(K(e1)-K(e2))/(e1-e2); divided
      // difference of K at x = e_m(k), y = -sg e_n(k'); one branch for the rare near-degenerate lanes
      T L[2][2];
      bool ok = true;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const T den = ekm[m] + sg * epn[n];
          ok = ok && nondegenerate<T, SCHEME>(den, ekm[m], sg * epn[n], lam);
          L[m][n] = sg * (Kkm[m] + sg * Kpn[n]) * rcp_fast(den);
        }
      if (__builtin_expect(!ok, 0)) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 2; ++n)
            L[m][n] = sg * divided_difference(ekm[m], -sg * epn[n], Kkm[m], -sg * Kpn[n], lam, dd_scheme(SCHEME),
                                              deriv);
      }
      if constexpr (SHELL) {
        // shell factor a_m(k) b_n(k') + b_m(k) a_n(k')
        const T ak[2] = {ck.cv.x, ck.cv.y}, bk[2] = {ck.cv.z, ck.cv.w};
        const T ap[2] = {cp.cv.x, cp.cv.y}, bp[2] = {cp.cv.z, cp.cv.w};
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 2; ++n) L[m][n] *= fma(ak[m], bp[n], bk[m] * ap[n]);
      }
      // W_1 = alpha_1 X_0 + L_11 1, D = W_0 - W_1 = (alpha_0 - alpha_1) X_0 + (L_01 - L_11) 1
      const T al0 = L[0][0] - L[0][1], al1 = L[1][0] - L[1][1];
      const T dal = al0 - al1, dl = L[0][1] - L[1][1];
      const T W1d0 = fma(al1, X0, L[1][1]), W1d1 = fma(al1, X1, L[1][1]);
      const T W1r = al1 * Xr, W1i = al1 * Xi;
      const T Dd0 = fma(dal, X0, dl), Dd1 = fma(dal, X1, dl);
      const T Dr = dal * Xr, Di = dal * Xi;
      // the 10 distinct entries of M = Pi_0 (x) D + 1 (x) W_1
      T mr[NREAL], mc[NCPLX][2];
      mr[0] = fma(P0, Dd0, W1d0);  // (0,0,0,0)
      mr[1] = fma(P0, Dd1, W1d1);  // (0,1,0,1)
      mr[2] = fma(P1, Dd0, W1d0);  // (1,0,1,0)
      mr[3] = fma(P1, Dd1, W1d1);  // (1,1,1,1)
      mc[0][0] = fma(P0, Dr, W1r);  // (0,0,0,1)
      mc[0][1] = fma(P0, Di, W1i);
      mc[1][0] = fma(P1, Dr, W1r);  // (1,0,1,1)
      mc[1][1] = fma(P1, Di, W1i);
      mc[2][0] = Pr * Dd0;  // (0,0,1,0)
      mc[2][1] = Pi * Dd0;
      mc[3][0] = Pr * Dd1;  // (0,1,1,1)
      mc[3][1] = Pi * Dd1;
      mc[4][0] = fma(Pr, Dr, -Pi * Di);  // (0,0,1,1): Pi_0[01] D[01]
      mc[4][1] = fma(Pr, Di, Pi * Dr);
      mc[5][0] = fma(Pr, Dr, Pi * Di);  // (0,1,1,0): Pi_0[01] D[10] = Pi_0[01] conj(D[01])
      mc[5][1] = fma(Pi, Dr, -Pr * Di);
#pragma unroll
      for (int t = 0; t < NREAL; ++t) Sr[t] += mr[t];
#pragma unroll
      for (int t = 0; t < NCPLX; ++t) {
        Sc[t][0] += mc[t][0];
        Sc[t][1] += mc[t][1];
      }
#pragma unroll
      for (int d = 0; d < NDX - 1; ++d) {
        const int j = jd[d];
        jd[d] = j + d + 1 >= Lf ? j + d + 1 - Lf : j + d + 1;
        const T c = twk[2 * j], s = twk[2 * j + 1];  // e^{-i 2 pi kx dx / Lf}, wave-uniform
#pragma unroll
        for (int t = 0; t < NREAL; ++t) {
          Ar[d][t] = fma(c, mr[t], Ar[d][t]);
          Br[d][t] = fma(s, mr[t], Br[d][t]);
        }
#pragma unroll
        for (int t = 0; t < NCPLX; ++t) {
          Ac[d][t][0] = fma(c, mc[t][0], Ac[d][t][0]);
          Ac[d][t][1] = fma(c, mc[t][1], Ac[d][t][1]);
          Bc[d][t][0] = fma(s, mc[t][0], Bc[d][t][0]);
          Bc[d][t][1] = fma(s, mc[t][1], Bc[d][t][1]);
        }
      }
  };
  const unsigned uky = (unsigned)ky, ukpy = (unsigned)kpy;
  if constexpr (sizeof(T) == 4 && NDX > 3) {
    // software pipeline with two register sets: the loads of point kx + 1 are
    // issued before the arithmetic of point kx; a prefetch past the chunk
    // re-reads the current point and is not used
    Pt ak, ap, bk, bp;
    load(x0, uky, ak);
    load(kpx, ukpy, ap);
    int kx = x0;
    for (; kx + 1 < x1; kx += 2) {
      next_kpx();
      load(kx + 1, uky, bk);
      load(kpx, ukpy, bp);
      point(ak, ap);
      const bool more = kx + 2 < x1;
      if (more) next_kpx();
      load(more ? kx + 2 : kx + 1, uky, ak);
      load(kpx, ukpy, ap);
      point(bk, bp);
    }
    if (kx < x1) point(ak, ap);
  } else {
    // plain order, one register set: FP32 with dx < 3 then fits four waves per
    // SIMD, which hide the load latency better than the second set did at three
    // (rashba_s9_L24: 2.26 -> 2.18 ms); FP64 is at one or two waves per SIMD anyway
    for (int kx = x0; kx < x1; ++kx) {
      Pt ck, cp;
      load(kx, uky, ck);
      load(kpx, ukpy, cp);
      point(ck, cp);
      next_kpx();
    }
  }
}

// A workgroup holds QW waves that share the ky block, q_x, kx chunk and
// channel and take QW consecutive q_y: they read the same k addresses and
// overlapping k -/+ q rows at the same time.  Workgroups are handed to the 8
// XCDs round-robin by linear id; each XCD is given a contiguous slice of the
// work items, ordered (ky block, q_y group, q_x, kx chunk, channel) from
// fastest to slowest, so that co-resident workgroups share rows in its L2.
constexpr int N_XCD = 8;

template <typename T>
struct loop_waves {
  static constexpr int v = (sizeof(T) == 4) ? 4 : 2;
};

// One work item (ky block, q_y group, q_x, kx chunk, channel) of QW waves,
// w its index among the n_items of one instance; bufs and phy are the
// workgroup's LDS.
template <typename T, int NDX, int NDY, int SCHEME, int QW>
__device__ __forceinline__ void loop_no2_item(const T *__restrict__ ekv, const T *__restrict__ pi4,
                                              const T *__restrict__ cvp, const double *__restrict__ tw,
                                              const T *__restrict__ twk, int Lq, int n_ref, int Lf, int nkyb,
                                              int nkxc, int kxper, int q_first, int n_q,
                                              const int *__restrict__ rows, int ch_first, int w, T lam, int deriv,
                                              T *__restrict__ partial, T (&bufs)[QW][32][65],
                                              T (&phy)[2 * NDY + 1][2][64]) {
  constexpr int NDY2 = 2 * NDY + 1;
  const int tid = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kyb = w % nkyb;
  w /= nkyb;
  const int nqyg = (Lq + QW - 1) / QW;
  const int qyg = w % nqyg;
  w /= nqyg;
  const bool qvalid = qyg * QW + wv < Lq;
  const int qy = qvalid ? qyg * QW + wv : Lq - 1;
  const int nqx = n_q / Lq;
  const int qx = w % nqx;
  w /= nqx;
  const int kxc = w % nkxc;
  const int chrel = w / nkxc, ch = ch_first + chrel;
  // coarse q: consecutive from q_first, or whole q_x rows from a list
  const int qrel = qx * Lq + qy, qi = rows ? rows[qx] * Lq + qy : q_first + qrel;
  const int nparts = nkyb * nkxc;
  // one coarse q per wave: keep its fine coordinates in scalar registers
  const int qfx = __builtin_amdgcn_readfirstlane((qi / Lq) * n_ref);
  const int qfy = __builtin_amdgcn_readfirstlane((qi % Lq) * n_ref);
  const int ky_raw = kyb * 64 + tid;
  const bool active = ky_raw < Lf;
  const int ky = active ? ky_raw : Lf - 1;
  const int x0 = kxc * kxper;
  const int x1 = min(Lf, x0 + kxper);

  // S: dx = 0 sums; A/B: sum of cos/sin parts for dx >= 1
  T Sr[NREAL], Sc[NCPLX][2], Ar[NDX - 1][NREAL], Br[NDX - 1][NREAL];
  T Ac[NDX - 1][NCPLX][2], Bc[NDX - 1][NCPLX][2];
#pragma unroll
  for (int t = 0; t < NREAL; ++t) Sr[t] = T(0);
#pragma unroll
  for (int t = 0; t < NCPLX; ++t) Sc[t][0] = Sc[t][1] = T(0);
#pragma unroll
  for (int d = 0; d < NDX - 1; ++d) {
#pragma unroll
    for (int t = 0; t < NREAL; ++t) Ar[d][t] = Br[d][t] = T(0);
#pragma unroll
    for (int t = 0; t < NCPLX; ++t) Ac[d][t][0] = Ac[d][t][1] = Bc[d][t][0] = Bc[d][t][1] = T(0);
  }
  if (ch == 0)
    loop_no2_body<T, NDX, SCHEME, 0>(ekv, pi4, cvp, twk, Lf, qfx, qfy, ky, x0, x1, lam, deriv, Sr, Sc, Ar, Br, Ac,
                                     Bc);
  else
    loop_no2_body<T, NDX, SCHEME, 1>(ekv, pi4, cvp, twk, Lf, qfx, qfy, ky, x0, x1, lam, deriv, Sr, Sc, Ar, Br, Ac,
                                     Bc);

  // rebuild all 16 entries per dx, transpose through LDS, contract with e^{-i 2 pi ky dy / Lf}
  T(&buf)[32][65] = bufs[wv];
  if (wv == 0) {
#pragma unroll
    for (int i = 0; i < NDY2; ++i) {
      int dy = i - NDY;
      int j = (int)(((long long)ky_raw * dy) % Lf);
      if (j < 0) j += Lf;
      phy[i][0][tid] = (T)tw[2 * j];
      phy[i][1][tid] = (T)tw[2 * j + 1];
    }
  }
  const T on = active ? T(1) : T(0);
  const size_t pbase = (((size_t)chrel * n_q + qrel) * nparts + (kyb + nkyb * kxc)) * (size_t)(NDX * NDY2 * 16);
#pragma unroll
  for (int dx = 0; dx < NDX; ++dx) {
    __syncthreads();
    if (dx == 0) {
#pragma unroll
      for (int t = 0; t < NREAL; ++t) {
        buf[2 * REAL_TAU[t]][tid] = on * Sr[t];
        buf[2 * REAL_TAU[t] + 1][tid] = T(0);
      }
#pragma unroll
      for (int t = 0; t < NCPLX; ++t) {
        buf[2 * CPLX_TAU[t]][tid] = on * Sc[t][0];
        buf[2 * CPLX_TAU[t] + 1][tid] = on * Sc[t][1];
        buf[2 * CPLX_PARTNER[t]][tid] = on * Sc[t][0];
        buf[2 * CPLX_PARTNER[t] + 1][tid] = -on * Sc[t][1];
      }
    } else {
      const int d = dx - 1;
#pragma unroll
      for (int t = 0; t < NREAL; ++t) {
        buf[2 * REAL_TAU[t]][tid] = on * Ar[d][t];
        buf[2 * REAL_TAU[t] + 1][tid] = on * Br[d][t];
      }
#pragma unroll
      for (int t = 0; t < NCPLX; ++t) {
        const T ar = Ac[d][t][0], ai = Ac[d][t][1], br = Bc[d][t][0], bi = Bc[d][t][1];
        buf[2 * CPLX_TAU[t]][tid] = on * (ar - bi);
        buf[2 * CPLX_TAU[t] + 1][tid] = on * (ai + br);
        buf[2 * CPLX_PARTNER[t]][tid] = on * (ar + bi);
        buf[2 * CPLX_PARTNER[t] + 1][tid] = on * (br - ai);
      }
    }
    __syncthreads();
    for (int o = tid; o < NDY2 * 16; o += 64) {
      const int t = o & 15;
      const int dyi = o >> 4;
      T sr = T(0), si = T(0);
#pragma unroll 4
      for (int l = 0; l < 64; ++l) {
        const T ar = buf[2 * t][l], ai = buf[2 * t + 1][l];
        const T pr = phy[dyi][0][l], pim = phy[dyi][1][l];
        sr = fma(pr, ar, sr);
        sr = fma(-pim, ai, sr);
        si = fma(pr, ai, si);
        si = fma(pim, ar, si);
      }
      const size_t idx = pbase + ((size_t)(dx * NDY2 + dyi) * 16 + t);
      if (qvalid) {
        partial[2 * idx] = sr;
        partial[2 * idx + 1] = si;
      }
    }
  }
}


// QW waves per work item (ky block, q_y group, q_x, kx chunk, channel).
template <typename T, int NDX, int NDY, int SCHEME, int QW>
__global__ __launch_bounds__(64 * QW, (NDX > 3 ? (sizeof(T) == 8 ? 1 : 2) : (sizeof(T) == 8 ? 2 : 4))) void loop_no2_kernel(const T *__restrict__ ekv, const T *__restrict__ pi4, const T *__restrict__ cvp,
                                                           const double *__restrict__ tw, const T *__restrict__ twk,
                                                           int Lq, int n_ref, int Lf,
                                                           int nkyb, int nkxc, int kxper, int q_first, int n_q,
                                                           const int *__restrict__ rows,
                                                           int ch_first, int n_items, T lam, int deriv,
                                                           T *__restrict__ partial) {
  __shared__ T bufs[QW][32][65];
  __shared__ T phy[2 * NDY + 1][2][64];
  const int xcd = blockIdx.x % N_XCD, slot = blockIdx.x / N_XCD;
  const int base = n_items / N_XCD, rem = n_items % N_XCD;
  if (slot >= base + (xcd < rem ? 1 : 0)) return;  // padding workgroup, no work
  const int w = xcd * base + min(xcd, rem) + slot;
  loop_no2_item<T, NDX, NDY, SCHEME, QW>(ekv, pi4, cvp, tw, twk, Lq, n_ref, Lf, nkyb, nkxc, kxper, q_first, n_q, rows,
                                         ch_first, w, lam, deriv, partial, bufs, phy);
}

// Several instances in one launch: the items of instance i are
// [inst[i].item0, inst[i].item0 + its count), every instance summing both
// channels over all its coarse q; the same work items and partial sums as its
// own launch.
template <typename T, int NDX, int NDY, int SCHEME, int QW>
__global__ __launch_bounds__(64 * QW, (NDX > 3 ? (sizeof(T) == 8 ? 1 : 2) : (sizeof(T) == 8 ? 2 : 4))) void loop_no2_batch_kernel(const No2Inst *__restrict__ inst, int n_inst, int n_items) {
  __shared__ T bufs[QW][32][65];
  __shared__ T phy[2 * NDY + 1][2][64];
  const int xcd = blockIdx.x % N_XCD, slot = blockIdx.x / N_XCD;
  const int base = n_items / N_XCD, rem = n_items % N_XCD;
  if (slot >= base + (xcd < rem ? 1 : 0)) return;  // padding workgroup, no work
  const int w = xcd * base + min(xcd, rem) + slot;
  int i = 0;
  while (i + 1 < n_inst && inst[i + 1].item0 <= w) ++i;
  const No2Inst &d = inst[i];
  loop_no2_item<T, NDX, NDY, SCHEME, QW>((const T *)d.ekv, (const T *)d.pi4, (const T *)d.cvp, d.tw,
                                         (const T *)d.twk, d.Lq, d.n_ref, d.Lf, d.nkyb, d.nkxc, d.kxper, 0, d.n_q,
                                         nullptr, 0, w - d.item0, (T)d.lam, d.deriv, (T *)d.partial, bufs, phy);
}

template <typename T, int NDX, int NDY>
static hipError_t launch_no2(const LoopArgs &a, hipStream_t st) {
  if (a.q_first % a.Lq != 0 || a.n_q % a.Lq != 0) return hipErrorInvalidValue;  // whole q_x rows
  constexpr int QW = loop_waves<T>::v;
  const int kxper = (a.Lf + a.nkxc - 1) / a.nkxc;
  const int nqyg = (a.Lq + QW - 1) / QW;
  const int n_items = a.nkyb * a.nkxc * nqyg * (a.n_q / a.Lq) * a.n_ch;
  const int n_wg = ((n_items + N_XCD - 1) / N_XCD) * N_XCD;
  dim3 grid(n_wg), block(64 * QW);
  const T *ekv = (const T *)a.ekv;
  const T *pi4 = (const T *)a.pi4;
  const T *twk = (const T *)(sizeof(T) == 8 ? (const void *)a.tw : a.tw32);
  const T *cvp = (const T *)a.cv;
  if (!ekv || !pi4 || !twk) return hipErrorInvalidValue;
  if (a.scheme == CUT_SHELL && !cvp) return hipErrorInvalidValue;
#define TUFRG_NO2_LAUNCH(S)                                                                                         \
  hipLaunchKernelGGL((loop_no2_kernel<T, NDX, NDY, S, QW>), grid, block, 0, st, ekv, pi4, cvp, a.tw, twk, a.Lq,    \
                     a.n_ref, a.Lf, a.nkyb, a.nkxc, kxper, a.q_first, a.n_q, a.rows, a.ch_first, n_items, (T)a.lam, \
                     a.deriv, (T *)a.partial)
  if (a.scheme == CUT_TEMPERATURE)
    TUFRG_NO2_LAUNCH(CUT_TEMPERATURE);
  else if (a.scheme == CUT_OMEGA)
    TUFRG_NO2_LAUNCH(CUT_OMEGA);
  else if (a.scheme == CUT_SHELL)
    TUFRG_NO2_LAUNCH(CUT_SHELL);
  else
    return hipErrorInvalidValue;
#undef TUFRG_NO2_LAUNCH
  return hipGetLastError();
}

template <typename T, int NDX, int NDY>
static hipError_t launch_no2_batch(const LoopArgs *a, const int *idx, int m, No2Inst *desc_h, No2Inst *desc_d,
                                   hipStream_t st) {
  constexpr int QW = loop_waves<T>::v;
  long long items = 0;
  for (int j = 0; j < m; ++j) {
    const LoopArgs &x = a[idx[j]];
    const T *twk = (const T *)(sizeof(T) == 8 ? (const void *)x.tw : x.tw32);
    if (!x.ekv || !x.pi4 || !twk || x.q_first != 0 || x.n_q != x.Nq || x.rows || x.ch_first != 0 || x.n_ch != 2)
      return hipErrorInvalidValue;
    if (x.scheme == CUT_SHELL && !x.cv) return hipErrorInvalidValue;
    No2Inst &d = desc_h[j];
    d.ekv = x.ekv;
    d.pi4 = x.pi4;
    d.cvp = x.cv;
    d.twk = twk;
    d.tw = x.tw;
    d.partial = x.partial;
    d.lam = x.lam;
    d.Lq = x.Lq;
    d.n_ref = x.n_ref;
    d.Lf = x.Lf;
    d.nkyb = x.nkyb;
    d.nkxc = x.nkxc;
    d.kxper = (x.Lf + x.nkxc - 1) / x.nkxc;
    d.n_q = x.n_q;
    d.deriv = x.deriv;
    d.item0 = (int)items;
    d.pad = 0;
    items += (long long)x.nkyb * x.nkxc * ((x.Lq + QW - 1) / QW) * (x.n_q / x.Lq) * 2;
  }
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyAsync(desc_d, desc_h, m * sizeof(No2Inst), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  const int n_items = (int)items;
  const dim3 grid(((n_items + N_XCD - 1) / N_XCD) * N_XCD), block(64 * QW);
  const int scheme = a[idx[0]].scheme;
  if (scheme == CUT_TEMPERATURE)
    hipLaunchKernelGGL((loop_no2_batch_kernel<T, NDX, NDY, CUT_TEMPERATURE, QW>), grid, block, 0, st, desc_d, m,
                       n_items);
  else if (scheme == CUT_OMEGA)
    hipLaunchKernelGGL((loop_no2_batch_kernel<T, NDX, NDY, CUT_OMEGA, QW>), grid, block, 0, st, desc_d, m, n_items);
  else if (scheme == CUT_SHELL)
    hipLaunchKernelGGL((loop_no2_batch_kernel<T, NDX, NDY, CUT_SHELL, QW>), grid, block, 0, st, desc_d, m, n_items);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_loop_batch(const LoopArgs *a, int n, No2Inst *desc_h, No2Inst *desc_d, hipStream_t st) {
  if (n < 1 || !desc_h || !desc_d) return hipErrorInvalidValue;
  const int prec = a[0].prec;
  for (int i = 0; i < n; ++i)
    if (a[i].n_o != 2 || a[i].prec != prec) return hipErrorInvalidValue;
  // one launch per (shape, regulator); the group's descriptors contiguous
  int off = 0;
  for (int shape = 0; shape < 3; ++shape)
    for (int scheme = 0; scheme < 3; ++scheme) {
      std::vector<int> idx;
      for (int i = 0; i < n; ++i) {
        const int sh = (a[i].ndx == 3 && a[i].ndy == 2) ? 0 : (a[i].ndx == 5 && a[i].ndy == 4) ? 1 : 2;
        if (sh == 2 && !(a[i].ndx == 2 && a[i].ndy == 1)) return hipErrorInvalidValue;
        if (sh == shape && a[i].scheme == scheme) idx.push_back(i);
      }
      if (idx.empty()) continue;
      const int m = (int)idx.size();
      hipError_t e;
      if (shape == 0)
        e = prec == 0 ? launch_no2_batch<double, 3, 2>(a, idx.data(), m, desc_h + off, desc_d + off, st)
                      : launch_no2_batch<float, 3, 2>(a, idx.data(), m, desc_h + off, desc_d + off, st);
      else if (shape == 1)
        e = prec == 0 ? launch_no2_batch<double, 5, 4>(a, idx.data(), m, desc_h + off, desc_d + off, st)
                      : launch_no2_batch<float, 5, 4>(a, idx.data(), m, desc_h + off, desc_d + off, st);
      else
        e = prec == 0 ? launch_no2_batch<double, 2, 1>(a, idx.data(), m, desc_h + off, desc_d + off, st)
                      : launch_no2_batch<float, 2, 1>(a, idx.data(), m, desc_h + off, desc_d + off, st);
      if (e != hipSuccess) return e;
      off += m;
    }
  return hipSuccess;
}

hipError_t launch_loop(const LoopArgs &a, hipStream_t st) {
  if (a.n_o == 6) return launch_loop_gen(a, st);
  if (a.n_o != 2) return hipErrorInvalidValue;
  const bool f64 = (a.prec == 0);
  if (a.ndx == 3 && a.ndy == 2) return f64 ? launch_no2<double, 3, 2>(a, st) : launch_no2<float, 3, 2>(a, st);
  if (a.ndx == 5 && a.ndy == 4) return f64 ? launch_no2<double, 5, 4>(a, st) : launch_no2<float, 5, 4>(a, st);
  if (a.ndx == 2 && a.ndy == 1) return f64 ? launch_no2<double, 2, 1>(a, st) : launch_no2<float, 2, 1>(a, st);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------

template <typename PT>
__global__ void loop_finalize_kernel(int n_o, int n_ch, int n_q, int nparts, int ndx, int ndy, int nD,
                                     const int *__restrict__ dlist, double inv_nf, const PT *__restrict__ partial,
                                     double *__restrict__ compact) {
  const int no2 = n_o * n_o, no4 = no2 * no2;
  const long long total = (long long)n_ch * n_q * nD * no4;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int tau = (int)(i % no4);
  const int iD = (int)((i / no4) % nD);
  const long long cq = i / ((long long)no4 * nD);  // chrel * n_q + qrel
  int dx = dlist[2 * iD], dy = dlist[2 * iD + 1];
  int t = tau;
  bool cj = false;
  if (dx < 0) {
    dx = -dx;
    dy = -dy;
    t = (tau % no2) * no2 + tau / no2;
    cj = true;
  }
  const int ndy2 = 2 * ndy + 1;
  const size_t per = (size_t)ndx * ndy2 * no4;
  const PT *p = partial + (size_t)cq * nparts * per * 2 + ((size_t)(dx * ndy2 + dy + ndy) * no4 + t) * 2;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < nparts; ++k) {
    sr += (double)p[(size_t)k * per * 2];
    si += (double)p[(size_t)k * per * 2 + 1];
  }
  compact[2 * i] = sr * inv_nf;
  compact[2 * i + 1] = (cj ? -si : si) * inv_nf;
}

hipError_t launch_loop_finalize(const LoopArgs &a, int nD, const int *dlist, double *compact, hipStream_t st) {
  const int no4 = a.n_o * a.n_o * a.n_o * a.n_o;
  const long long total = (long long)a.n_ch * a.n_q * nD * no4;
  const int nparts = a.nkyb * a.nkxc;
  const double inv = 1.0 / ((double)a.Lf * a.Lf);
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (a.prec == 0)
    hipLaunchKernelGGL(loop_finalize_kernel<double>, grid, block, 0, st, a.n_o, a.n_ch, a.n_q, nparts, a.ndx, a.ndy,
                       nD, dlist, inv, (const double *)a.partial, compact);
  else
    hipLaunchKernelGGL(loop_finalize_kernel<float>, grid, block, 0, st, a.n_o, a.n_ch, a.n_q, nparts, a.ndx, a.ndy,
                       nD, dlist, inv, (const float *)a.partial, compact);
  return hipGetLastError();
}

__global__ void loop_expand_kernel(int n_o, int n_ff, int nD, int n_q, const int *__restrict__ didx,
                                   const double *__restrict__ compact, double *__restrict__ out) {
  const int no2 = n_o * n_o, no4 = no2 * no2;
  const int B = n_ff * no2;
  const long long total = (long long)n_q * B * B;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int col = (int)(i % B), row = (int)((i / B) % B);
  const long long q = i / ((long long)B * B);
  const int r1 = row / no2, ab = row % no2, r2 = col / no2, cd = col % no2;
  const int iD = didx[r1 * n_ff + r2];
  const size_t src = ((size_t)q * nD + iD) * no4 + (size_t)ab * no2 + cd;
  out[2 * i] = compact[2 * src];
  out[2 * i + 1] = compact[2 * src + 1];
}

hipError_t launch_loop_expand(int n_o, int n_ff, int nD, int n_q, const int *didx, const double *compact,
                              double *out, hipStream_t st) {
  const int B = n_ff * n_o * n_o;
  const long long total = (long long)n_q * B * B;
  hipLaunchKernelGGL(loop_expand_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n_o, n_ff, nD,
                     n_q, didx, compact, out);
  return hipGetLastError();
}

}  // namespace tufrg

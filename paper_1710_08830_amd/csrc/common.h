// Device-side helpers of the TU-fRG library: complex arithmetic and the
// regulator functions whose divided differences are the loop kernels.
//
// Loops (Sec. 3.1 of the paper, generalised to the temperature and Omega
// regulators): with an odd function J_Lambda(e) and K = dJ/dLambda,
//   L-(e1, e2) =  (K(e1) + K(e2)) / (e1 + e2)    (particle-particle)
//   L+(e1, e2) = -(K(e1) - K(e2)) / (e1 - e2)    (particle-hole)
// Temperature flow (Lambda = T): J = tanh(e / 2T) / 2, the Fermi-function
// combination 1 - 2 f(e).  Omega scheme at T = 0 (propagator times
// w^2 / (w^2 + Omega^2)): J = e (2|e| + Omega) / (4 (|e| + Omega)^2).
// At coinciding arguments the divided difference is the mean of K' over the
// interval (two-point Gauss-Legendre, split at e = 0 for the Omega scheme).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tufrg {

enum { CUT_TEMPERATURE = 0, CUT_OMEGA = 1, CUT_SHELL = 2 };

// The momentum-shell scheme (Sec. 3.1 regulator) takes its bubbles at a fixed
// temperature: its divided differences are those of the temperature scheme,
// evaluated at Lambda = T, and the loop kernels carry a shell factor.
__host__ __device__ constexpr int dd_scheme(int scheme) { return scheme == CUT_SHELL ? CUT_TEMPERATURE : scheme; }

// Shell factor of a band value: the loop kernel of a pair is the fixed-T
// divided difference times a_m b_n + b_m a_n, with chi = e^2 / (e^2 + Lambda^2)
// and (a, b) = (d chi / d Lambda, chi) for the loop (deriv) or
// (chi, chi) / sqrt 2 for the bubble.
template <typename T>
__device__ inline void shell_ab(T e, T lam, int deriv, T &a, T &b) {
  const T e2 = e * e, d = e2 + lam * lam;
  const T chi = e2 / d;
  if (deriv) {
    a = -T(2) * lam * e2 / (d * d);
    b = chi;
  } else {
    a = b = chi * T(0.70710678118654752440);
  }
}

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__host__ __device__ inline cx<T> cmake(T r, T i) {
  cx<T> z;
  z.re = r;
  z.im = i;
  return z;
}

template <typename T>
__host__ __device__ inline cx<T> cadd(cx<T> a, cx<T> b) {
  return cmake(a.re + b.re, a.im + b.im);
}

template <typename T>
__host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return cmake(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}

// acc += a * b
template <typename T>
__host__ __device__ inline void cfma(cx<T> &acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}

// acc += a * conj(b)
template <typename T>
__host__ __device__ inline void cfmaconj(cx<T> &acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.im, b.re, acc.im);
  acc.im = fma(-a.re, b.im, acc.im);
}

// Fast reciprocal: hardware estimate refined by Newton steps (FP64) or the
// 1-ulp hardware reciprocal (FP32).
__device__ inline double rcp_fast(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  return r;
}
__device__ inline float rcp_fast(float d) { return __builtin_amdgcn_rcpf(d); }

// sech^2(x) and tanh(x) from s = exp(-2|x|), stable for every x.
// 1 / x: exact division in FP64, the hardware reciprocal in FP32
__device__ inline double rdiv(double x) { return 1.0 / x; }
__device__ inline float rdiv(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ inline void sech2_tanh(T x, T &sech2, T &th) {
  T ax = fabs(x);
  T s = exp(T(-2) * ax);
  T inv = T(1) / (T(1) + s);
  sech2 = T(4) * s * inv * inv;
  th = copysign((T(1) - s) * inv, x);
}

// J or K = dJ/dLambda at energy e (deriv selects K).
template <typename T>
__device__ inline T cut_val(T e, T lam, int scheme, int deriv) {
  if (scheme == CUT_TEMPERATURE) {
    T x = e / (T(2) * lam);
    T s2, th;
    sech2_tanh(x, s2, th);
    if (deriv) return -e * s2 / (T(4) * lam * lam);
    return T(0.5) * th;
  }
  T a = fabs(e);
  T d = a + lam;
  if (deriv) return -e * (T(3) * a + lam) * rdiv(T(4) * d * d * d);
  return e * (T(2) * a + lam) * rdiv(T(4) * d * d);
}

// d/de of cut_val.
template <typename T>
__device__ inline T cut_der(T e, T lam, int scheme, int deriv) {
  if (scheme == CUT_TEMPERATURE) {
    T x = e / (T(2) * lam);
    T s2, th;
    sech2_tanh(x, s2, th);
    if (deriv) return -s2 * (T(1) - T(2) * x * th) / (T(4) * lam * lam);
    return s2 / (T(4) * lam);
  }
  T a = fabs(e);
  T d = a + lam;
  T d2 = d * d;
  if (deriv) return (T(3) * e * e - T(4) * a * lam - lam * lam) * rdiv(T(4) * d2 * d2);
  return lam * (T(3) * a + lam) * rdiv(T(4) * d2 * d);
}

template <typename T>
__device__ inline T gl2_mean(T a, T b, T lam, int scheme, int deriv) {
  const T c = T(0.57735026918962576451);  // 1/sqrt(3)
  T m = T(0.5) * (a + b), h = T(0.5) * (b - a);
  return T(0.5) * (cut_der(m - c * h, lam, scheme, deriv) + cut_der(m + c * h, lam, scheme, deriv));
}

// Relative width below which the divided difference switches to the mean of
// the derivative.  FP64: 1e-3; FP32: 2e-2 (cancellation in the quotient costs
// about eps / width = 3e-6 at the switch, the two-point rule (width / 2)^4 /
// 135; a wider switch sends more lanes, and with them whole waves, through the
// slower branch: at 5e-2 the Rashba loop ran 6 % slower with the same error).
template <typename T>
struct degen_rel;
template <>
struct degen_rel<double> {
  static constexpr double v = 1e-3;
};
template <>
struct degen_rel<float> {
  static constexpr float v = 2e-2f;
};

// (g(x) - g(y)) / (x - y) given gx = g(x), gy = g(y).
template <typename T>
__device__ inline T divided_difference(T x, T y, T gx, T gy, T lam, int scheme, int deriv) {
  T d = x - y;
  T scale = (scheme == CUT_TEMPERATURE) ? lam : lam + fabs(x) + fabs(y);
  if (fabs(d) > degen_rel<T>::v * scale) return (gx - gy) * rcp_fast(d);
  if (scheme == CUT_OMEGA && x * y < T(0)) {
    T w1 = fabs(x) / (fabs(x) + fabs(y));
    return w1 * gl2_mean(x, T(0), lam, scheme, deriv) +
           (T(1) - w1) * gl2_mean(T(0), y, lam, scheme, deriv);
  }
  return gl2_mean(x, y, lam, scheme, deriv);
}

}  // namespace tufrg

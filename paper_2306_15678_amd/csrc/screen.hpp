// screen.hpp -- pointwise nonlinear screen of one split step and its adjoint.
//
// Device units: u = U / sqrt(I_a), x = |u|^2 = I / I_a.  With
// cK = k0 n2 I_a dz and cM = (K-1) beta_K I_a^(K-1) dz the screen of one
// step (Eq. (1) Kerr, Eq. (3) plasma refraction and multiphoton absorption,
// Eq. (9) ansatz and turbulence) is E(x) = A(x) exp(i Phi(x)):
//   Phi = cK x                                        (Kerr)
//       - cK x^K / (1 + x^(K-1))                       (saturating plasma)
//       + cK Re f(x)                                   (ansatz)
//   ln A = -ln(1 + cM x^(K-1)) / (2(K-1))              (exact pointwise MPA)
//        - cK Im f(x)                                  (ansatz)
//   f(x) = [sum_p th_p x^p + i sum_p th_{4+p} x^p] / (1 + x^4)
// and a turbulence phase phi_t (a precomputed plane) on screen steps.
//
// The adjoint of w = V E(|V|^2) for a real loss, with G = dL/dRe + i dL/dIm:
//   G_V = G_w conj(E) (1 + x conj(g)) + conj(G_w) V^2 E g,   g = E'(x)/E(x)
//   g   = (ln A)'(x) + i Phi'(x)
// and the ansatz gradient dL/dth_p = Re(conj(G_w) w dlnE/dth_p), where
// dlnE/dth_p = i cK x^p/(1+x^4) (p <= 4) and -cK x^(p-4)/(1+x^4) (p > 4).
#pragma once

#include "fft_core.hpp"

namespace ssfm {

enum : unsigned {
  T_KERR = 1u,
  T_MPA = 2u,
  T_PLASMA = 4u,
  T_ANSATZ = 8u,
  T_TURB = 16u,
  T_PRECISE = 1u << 8  // FP32: library sincosf instead of v_sin/v_cos
};

template <typename R>
struct ScreenConst {
  R cK, cM, inv2k1;  // inv2k1 = 1 / (2 (K - 1))
  R th[8];
  int K;
  unsigned terms;
};

// x^m for the multiphoton exponents; K = 8 (m = 7, 6) is the air model and
// takes a short multiply chain (uniform branch), other orders the loop.
template <typename R>
__device__ __forceinline__ R ipow(R x, int m) {
  if (m == 7) {
    const R x2 = x * x, x4 = x2 * x2;
    return x4 * x2 * x;
  }
  if (m == 6) {
    const R x2 = x * x;
    return x2 * x2 * x2;
  }
  R r = R(1);
  for (int i = 0; i < m; ++i) r *= x;
  return r;
}

// FP32: hardware transcendentals (v_log_f32, v_exp_f32, v_rcp_f32 and
// v_sin_f32 / v_cos_f32, which take their argument in revolutions).  The
// phase is reduced to [-1/2, 1/2] revolutions first, so the hardware sine
// sees a small argument; the reduction costs one multiply and one rint.
// FP64 uses the device math library throughout.
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double fast_log2(double x) { return log2(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double fast_exp2(double x) { return exp2(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ void sin_cos(float a, float* s, float* c, bool precise) {
  if (precise) {
    sincosf(a, s, c);
    return;
  }
  float r = a * 0.15915494309189533577f;  // radians -> revolutions
  r -= rintf(r);
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void sin_cos(double a, double* s, double* c, bool) { sincos(a, s, c); }

// ln A and Phi (without turbulence) at x.
template <typename R>
__device__ __forceinline__ void screen_eval(const ScreenConst<R>& s, R x,
                                            R& log_a, R& phi) {
  log_a = R(0);
  phi = R(0);
  const unsigned tm = s.terms;
  R xk1 = R(0);
  if (tm & (T_MPA | T_PLASMA)) xk1 = ipow(x, s.K - 1);
  if (tm & T_KERR) phi += s.cK * x;
  // x^K/(1+x^(K-1)) written as x (1 - 1/(1+x^(K-1))): finite for any x
  if (tm & T_PLASMA) phi -= s.cK * x * (R(1) - rcp(R(1) + xk1));
  if (tm & T_MPA) {
    // ln A = -log2(1 + cM x^(K-1)) ln2 / (2(K-1))
    log_a -= fast_log2(R(1) + s.cM * xk1) * (R(0.69314718055994530942) * s.inv2k1);
  }
  if (tm & T_ANSATZ) {
    const R x2 = x * x, x3 = x2 * x, x4 = x2 * x2;
    const R inv = rcp(R(1) + x4);
    const R re = (s.th[0] * x + s.th[1] * x2 + s.th[2] * x3 + s.th[3] * x4) * inv;
    const R im = (s.th[4] * x + s.th[5] * x2 + s.th[6] * x3 + s.th[7] * x4) * inv;
    phi += s.cK * re;
    log_a -= s.cK * im;
  }
}

// A^2 at x (for the power diagnostics: |E V|^2 = x A^2).
template <typename R>
__device__ __forceinline__ R screen_amp2(const ScreenConst<R>& s, R x) {
  const unsigned tm = s.terms;
  R l2 = R(0);  // log2 of A^2
  if (tm & T_MPA) {
    const R xk1 = ipow(x, s.K - 1);
    l2 -= fast_log2(R(1) + s.cM * xk1) * (R(2) * s.inv2k1);
  }
  if (tm & T_ANSATZ) {
    const R x2 = x * x, x3 = x2 * x, x4 = x2 * x2;
    const R im = (s.th[4] * x + s.th[5] * x2 + s.th[6] * x3 + s.th[7] * x4) *
                 rcp(R(1) + x4);
    l2 -= R(2) * s.cK * im * R(1.44269504088896340736);
  }
  if (l2 == R(0)) return R(1);
  return fast_exp2(l2);
}

// u <- u E(|u|^2) exp(i phi_t)
template <typename R>
__device__ __forceinline__ cx<R> screen_apply(const ScreenConst<R>& s, cx<R> u,
                                              R phi_t) {
  const R x = u.re * u.re + u.im * u.im;
  R log_a, phi;
  screen_eval(s, x, log_a, phi);
  phi += phi_t;
  const R a = (log_a == R(0)) ? R(1) : fast_exp2(log_a * R(1.44269504088896340736));
  R sn, cs;
  sin_cos(phi, &sn, &cs, (s.terms & T_PRECISE) != 0);
  return {a * (u.re * cs - u.im * sn), a * (u.re * sn + u.im * cs)};
}

// Adjoint of the screen at the point V (pre-screen value).  lam is the
// cotangent of the screened value (after turbulence).  Returns the
// cotangent of V and adds the ansatz gradient terms to gth[8].
template <typename R>
__device__ __forceinline__ cx<R> screen_adjoint(const ScreenConst<R>& s,
                                                cx<R> v, cx<R> lam, R phi_t,
                                                double* gth) {
  const unsigned tm = s.terms;
  if (phi_t != R(0)) {  // lam <- conj(T) lam
    R sn, cs;
    sin_cos(phi_t, &sn, &cs, (tm & T_PRECISE) != 0);
    lam = {lam.re * cs + lam.im * sn, lam.im * cs - lam.re * sn};
  }
  const R x = v.re * v.re + v.im * v.im;
  R log_a = R(0), phi = R(0), dla = R(0), dphi = R(0);
  R xk1 = R(0), xk2 = R(0);
  if (tm & (T_MPA | T_PLASMA)) {
    xk2 = ipow(x, s.K - 2);
    xk1 = xk2 * x;
  }
  if (tm & T_KERR) {
    phi += s.cK * x;
    dphi += s.cK;
  }
  if (tm & T_PLASMA) {
    // with id = 1/(1+x^(K-1)): x^(K-1) id = 1 - id (no overflow at large x)
    const R id = rcp(R(1) + xk1);
    const R sat = R(1) - id;
    phi -= s.cK * x * sat;
    dphi -= s.cK * sat * (R(s.K) * id + sat);
  }
  if (tm & T_MPA) {
    const R q = R(1) + s.cM * xk1;
    log_a -= fast_log2(q) * (R(0.69314718055994530942) * s.inv2k1);
    dla -= s.cM * xk2 * R(0.5) * rcp(q);
  }
  R bx[4] = {R(0), R(0), R(0), R(0)};
  if (tm & T_ANSATZ) {
    const R x2 = x * x, x3 = x2 * x, x4 = x2 * x2;
    const R inv = rcp(R(1) + x4);
    const R gre = s.th[0] * x + s.th[1] * x2 + s.th[2] * x3 + s.th[3] * x4;
    const R gim = s.th[4] * x + s.th[5] * x2 + s.th[6] * x3 + s.th[7] * x4;
    const R dgre = s.th[0] + R(2) * s.th[1] * x + R(3) * s.th[2] * x2 + R(4) * s.th[3] * x3;
    const R dgim = s.th[4] + R(2) * s.th[5] * x + R(3) * s.th[6] * x2 + R(4) * s.th[7] * x3;
    const R d4 = R(4) * x3 * inv;
    const R re = gre * inv, im = gim * inv;
    phi += s.cK * re;
    log_a -= s.cK * im;
    dphi += s.cK * (dgre * inv - re * d4);
    dla -= s.cK * (dgim * inv - im * d4);
    bx[0] = x * inv;
    bx[1] = x2 * inv;
    bx[2] = x3 * inv;
    bx[3] = x4 * inv;
  }
  const R a = (log_a == R(0)) ? R(1) : fast_exp2(log_a * R(1.44269504088896340736));
  R sn, cs;
  sin_cos(phi, &sn, &cs, (tm & T_PRECISE) != 0);
  const cx<R> e = {a * cs, a * sn};
  // 1 + x conj(g), g = dla + i dphi
  const cx<R> one_xg = {R(1) + x * dla, -x * dphi};
  const cx<R> t1 = cmul(cmulc(lam, e), one_xg);  // lam conj(E) (1 + x conj g)
  const cx<R> v2 = {v.re * v.re - v.im * v.im, R(2) * v.re * v.im};
  const cx<R> eg = cmul(e, cx<R>{dla, dphi});
  const cx<R> t2 = cmul(cmul(conjg(lam), v2), eg);  // conj(lam) V^2 E g
  if (tm & T_ANSATZ) {
    // q = conj(lam) w, w = V E
    const cx<R> w = cmul(v, e);
    const R q_re = lam.re * w.re + lam.im * w.im;
    const R q_im = lam.re * w.im - lam.im * w.re;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      gth[p] += -double(s.cK) * double(q_im) * double(bx[p]);
      gth[4 + p] += -double(s.cK) * double(q_re) * double(bx[p]);
    }
  }
  return t1 + t2;
}

// ------------------------------------------------------------------------
// Batched forms over C points of one thread.  The term tests are uniform
// over a launch; here they sit outside the point loops, so a thread takes
// each branch once per batch instead of once per point.  Per point the
// arithmetic and its order are those of the single-point forms above.

template <typename R, int C>
__device__ __forceinline__ void ipow_n(const R* x, int m, R* out) {
  if (m == 7) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const R x2 = x[e] * x[e], x4 = x2 * x2;
      out[e] = x4 * x2 * x[e];
    }
  } else if (m == 6) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const R x2 = x[e] * x[e];
      out[e] = x2 * x2 * x2;
    }
  } else {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      R r = R(1);
      for (int i = 0; i < m; ++i) r *= x[e];
      out[e] = r;
    }
  }
}

// ln A and Phi (without turbulence) at C points.
template <typename R, int C>
__device__ __forceinline__ void screen_eval_n(const ScreenConst<R>& s, const R* x, R* log_a,
                                              R* phi) {
  const unsigned tm = s.terms;
#pragma unroll
  for (int e = 0; e < C; ++e) {
    log_a[e] = R(0);
    phi[e] = R(0);
  }
  R xk1[C];
  if (tm & (T_MPA | T_PLASMA)) ipow_n<R, C>(x, s.K - 1, xk1);
  if (tm & T_KERR) {
#pragma unroll
    for (int e = 0; e < C; ++e) phi[e] += s.cK * x[e];
  }
  if (tm & T_PLASMA) {
#pragma unroll
    for (int e = 0; e < C; ++e) phi[e] -= s.cK * x[e] * (R(1) - rcp(R(1) + xk1[e]));
  }
  if (tm & T_MPA) {
#pragma unroll
    for (int e = 0; e < C; ++e)
      log_a[e] -= fast_log2(R(1) + s.cM * xk1[e]) * (R(0.69314718055994530942) * s.inv2k1);
  }
  if (tm & T_ANSATZ) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const R xe = x[e], x2 = xe * xe, x3 = x2 * xe, x4 = x2 * x2;
      const R inv = rcp(R(1) + x4);
      const R re = (s.th[0] * xe + s.th[1] * x2 + s.th[2] * x3 + s.th[3] * x4) * inv;
      const R im = (s.th[4] * xe + s.th[5] * x2 + s.th[6] * x3 + s.th[7] * x4) * inv;
      phi[e] += s.cK * re;
      log_a[e] -= s.cK * im;
    }
  }
}

// A^2 at C points.
template <typename R, int C>
__device__ __forceinline__ void screen_amp2_n(const ScreenConst<R>& s, const R* x, R* out) {
  const unsigned tm = s.terms;
  R l2[C];
#pragma unroll
  for (int e = 0; e < C; ++e) l2[e] = R(0);
  if (tm & T_MPA) {
    R xk1[C];
    ipow_n<R, C>(x, s.K - 1, xk1);
#pragma unroll
    for (int e = 0; e < C; ++e)
      l2[e] -= fast_log2(R(1) + s.cM * xk1[e]) * (R(2) * s.inv2k1);
  }
  if (tm & T_ANSATZ) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const R xe = x[e], x2 = xe * xe, x3 = x2 * xe, x4 = x2 * x2;
      const R im = (s.th[4] * xe + s.th[5] * x2 + s.th[6] * x3 + s.th[7] * x4) *
                   rcp(R(1) + x4);
      l2[e] -= R(2) * s.cK * im * R(1.44269504088896340736);
    }
  }
  if (tm & (T_MPA | T_ANSATZ)) {
#pragma unroll
    for (int e = 0; e < C; ++e) out[e] = (l2[e] == R(0)) ? R(1) : fast_exp2(l2[e]);
  } else {
#pragma unroll
    for (int e = 0; e < C; ++e) out[e] = R(1);
  }
}

// u <- u E(|u|^2) exp(i phi_t) at C points.
template <typename R, int C>
__device__ __forceinline__ void screen_apply_n(const ScreenConst<R>& s, cx<R>* u,
                                               const R* phi_t) {
  R x[C], log_a[C], phi[C];
#pragma unroll
  for (int e = 0; e < C; ++e) x[e] = u[e].re * u[e].re + u[e].im * u[e].im;
  screen_eval_n<R, C>(s, x, log_a, phi);
  R a[C];
  if (s.terms & (T_MPA | T_ANSATZ)) {
#pragma unroll
    for (int e = 0; e < C; ++e)
      a[e] = (log_a[e] == R(0)) ? R(1) : fast_exp2(log_a[e] * R(1.44269504088896340736));
  } else {
#pragma unroll
    for (int e = 0; e < C; ++e) a[e] = R(1);
  }
  R sn[C], cs[C];
  if (s.terms & T_PRECISE) {
#pragma unroll
    for (int e = 0; e < C; ++e) sin_cos(phi[e] + phi_t[e], &sn[e], &cs[e], true);
  } else {
#pragma unroll
    for (int e = 0; e < C; ++e) sin_cos(phi[e] + phi_t[e], &sn[e], &cs[e], false);
  }
#pragma unroll
  for (int e = 0; e < C; ++e)
    u[e] = {a[e] * (u[e].re * cs[e] - u[e].im * sn[e]),
            a[e] * (u[e].re * sn[e] + u[e].im * cs[e])};
}

// Adjoint of the screen at C points (see screen_adjoint): lam holds the
// cotangents of the screened values and is overwritten with those of V;
// the ansatz gradient terms are added to gth[8] point by point in order.
// has_plane: a turbulence plane phi_t is applied at this step.
// SERIAL: a scheduling barrier after each point's gradient terms, so the
// FP64 products of later points are not computed ahead and held.
template <typename R, int C, bool SERIAL = false>
__device__ __forceinline__ void screen_adjoint_n(const ScreenConst<R>& s, const cx<R>* v,
                                                 cx<R>* lam, const R* phi_t, bool has_plane,
                                                 double* gth) {
  const unsigned tm = s.terms;
  const bool precise = (tm & T_PRECISE) != 0;
  if (has_plane) {  // lam <- conj(T) lam
#pragma unroll
    for (int e = 0; e < C; ++e) {
      R sn, cs;
      sin_cos(phi_t[e], &sn, &cs, precise);
      lam[e] = {lam[e].re * cs + lam[e].im * sn, lam[e].im * cs - lam[e].re * sn};
    }
  }
  R x[C], log_a[C], phi[C], dla[C], dphi[C];
#pragma unroll
  for (int e = 0; e < C; ++e) {
    x[e] = v[e].re * v[e].re + v[e].im * v[e].im;
    log_a[e] = phi[e] = dla[e] = dphi[e] = R(0);
  }
  R xk1[C], xk2[C];
  if (tm & (T_MPA | T_PLASMA)) {
    ipow_n<R, C>(x, s.K - 2, xk2);
#pragma unroll
    for (int e = 0; e < C; ++e) xk1[e] = xk2[e] * x[e];
  }
  if (tm & T_KERR) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      phi[e] += s.cK * x[e];
      dphi[e] += s.cK;
    }
  }
  if (tm & T_PLASMA) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const R id = rcp(R(1) + xk1[e]);
      const R sat = R(1) - id;
      phi[e] -= s.cK * x[e] * sat;
      dphi[e] -= s.cK * sat * (R(s.K) * id + sat);
    }
  }
  if (tm & T_MPA) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const R q = R(1) + s.cM * xk1[e];
      log_a[e] -= fast_log2(q) * (R(0.69314718055994530942) * s.inv2k1);
      dla[e] -= s.cM * xk2[e] * R(0.5) * rcp(q);
    }
  }
  const bool ansatz = (tm & T_ANSATZ) != 0;
  R inv_a[C];
  if (ansatz) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const R xe = x[e], x2 = xe * xe, x3 = x2 * xe, x4 = x2 * x2;
      const R inv = rcp(R(1) + x4);
      inv_a[e] = inv;
      const R gre = s.th[0] * xe + s.th[1] * x2 + s.th[2] * x3 + s.th[3] * x4;
      const R gim = s.th[4] * xe + s.th[5] * x2 + s.th[6] * x3 + s.th[7] * x4;
      const R dgre = s.th[0] + R(2) * s.th[1] * xe + R(3) * s.th[2] * x2 + R(4) * s.th[3] * x3;
      const R dgim = s.th[4] + R(2) * s.th[5] * xe + R(3) * s.th[6] * x2 + R(4) * s.th[7] * x3;
      const R d4 = R(4) * x3 * inv;
      const R re = gre * inv, im = gim * inv;
      phi[e] += s.cK * re;
      log_a[e] -= s.cK * im;
      dphi[e] += s.cK * (dgre * inv - re * d4);
      dla[e] -= s.cK * (dgim * inv - im * d4);
    }
  }
  R sn[C], cs[C];
  if (precise) {
#pragma unroll
    for (int e = 0; e < C; ++e) sin_cos(phi[e], &sn[e], &cs[e], true);
  } else {
#pragma unroll
    for (int e = 0; e < C; ++e) sin_cos(phi[e], &sn[e], &cs[e], false);
  }
#pragma unroll
  for (int e = 0; e < C; ++e) {
    const R a = (log_a[e] == R(0)) ? R(1) : fast_exp2(log_a[e] * R(1.44269504088896340736));
    const cx<R> ee = {a * cs[e], a * sn[e]};
    // 1 + x conj(g), g = dla + i dphi
    const cx<R> one_xg = {R(1) + x[e] * dla[e], -x[e] * dphi[e]};
    const cx<R> t1 = cmul(cmulc(lam[e], ee), one_xg);
    const cx<R> v2 = {v[e].re * v[e].re - v[e].im * v[e].im, R(2) * v[e].re * v[e].im};
    const cx<R> eg = cmul(ee, cx<R>{dla[e], dphi[e]});
    const cx<R> t2 = cmul(cmul(conjg(lam[e]), v2), eg);
    if (ansatz) {
      const R xe = x[e], x2 = xe * xe, x3 = x2 * xe, x4 = x2 * x2;
      const R inv = inv_a[e];
      const R bx[4] = {xe * inv, x2 * inv, x3 * inv, x4 * inv};
      const cx<R> w = cmul(v[e], ee);
      const R q_re = lam[e].re * w.re + lam[e].im * w.im;
      const R q_im = lam[e].re * w.im - lam[e].im * w.re;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        gth[p] += -double(s.cK) * double(q_im) * double(bx[p]);
        gth[4 + p] += -double(s.cK) * double(q_re) * double(bx[p]);
      }
    }
    lam[e] = t1 + t2;
    if constexpr (SERIAL) __builtin_amdgcn_sched_barrier(0);
  }
}

}  // namespace ssfm

// lens_vjp.hpp -- vector-Jacobian product of the effective-lens screen
// (Eq. (4)-(6)): the cotangent of the lens input and the gradients of the
// lens parameters, for fitting the lens by gradients.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace ssfm {

// gradient slots: c1, c2, then (amplitude, frequency, phase) of the 8 real
// segments, then of the 8 imaginary ones
constexpr int kLensGrads = 2 + 3 * 16;

// wk[i] = (|u[i]|^2 / i_ref, 0) for one beam's n2 points (u: complex128 SI).
template <typename R>
hipError_t launch_lens_vjp_prep(const double* u, double i_ref, void* wk, int64_t n2,
                                hipStream_t st);
// Per point (wk: filtered intensity in): g_in = conj(E) g_out, wk <- h I_a,
// per-block parameter partials into part[blocks][kLensGrads].
template <typename R>
hipError_t launch_lens_vjp_point(const double* u, const double* g_out, void* wk, double* g_in,
                                 int64_t n2, const LensDev& p, double* part, hipStream_t st);
// g_in += 2 Gauss(h) u (wk: the filtered h I_a), then grads[kLensGrads] =
// fixed-order sums of the partials.
template <typename R>
hipError_t launch_lens_vjp_final(const double* u, const void* wk, double i_ref, double* g_in,
                                 int64_t n2, double* part, double* grads, hipStream_t st);
// blocks of the point kernel (partials rows)
int lens_vjp_blocks(int64_t n2);

}  // namespace ssfm

// subharmonics.hpp -- low-frequency part of the turbulence screens by the
// subharmonic method (Lane, Glindemann and Dainty, Waves in Random Media 2
// (1992) 209), added to the FFT screens after their inverse transform.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace ssfm {

constexpr int kMaxSubharmonicLevels = 8;
// offset (in doubles) of the axis tables in a pair's scratch, after the
// 8 kMaxSubharmonicLevels coefficients (re, im) and the mean
constexpr int kSubTab = 256;

// Spectrum of one beam's subharmonic modes: kind 0 Kolmogorov with Fried
// parameter r0, kind 1 the step spectrum (tau per FFT cell, i.e. density
// tau L^2, inside kappa^2 <= kappa_h^2).
struct SubharmonicSpec {
  int32_t levels;
  int32_t kind;
  double r0;
  double tau;
  double kappa_h;
  double length;
};

// Adds the subharmonic part of screen pair `pair` of beam b to its screen
// planes (real part to plane 2 pair, imaginary part to plane 2 pair + 1 when
// the beam has it).  1 <= spec.levels <= kMaxSubharmonicLevels.  scratch:
// device memory of at least subharmonic_scratch_bytes(n, levels) bytes,
// 8-byte aligned (coefficients, mean and axis tables of this pair).
template <typename R>
hipError_t launch_subharmonics(const InstDev* inst, int b, int n, int pair, uint64_t seed,
                               const SubharmonicSpec& spec, void* planes, void* scratch,
                               hipStream_t s);

inline size_t subharmonic_scratch_bytes(int n, int levels) {
  return sizeof(double) * (kSubTab + 2 * size_t(levels) * size_t(n));
}

}  // namespace ssfm

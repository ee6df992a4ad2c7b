// subharmonics.hpp -- low-frequency part of the turbulence screens by the
// subharmonic method (Lane, Glindemann and Dainty, Waves in Random Media 2
// (1992) 209), added to the FFT screens after their inverse transform.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace ssfm {

constexpr int kMaxSubharmonicLevels = 8;
// doubles per screen pair's coefficient block: the 8 kMaxSubharmonicLevels
// coefficients (re, im) at [0, 128), the grid mean at [128, 130)
constexpr int kSubPair = 256;

// Spectrum of one beam's subharmonic modes: kind 0 Kolmogorov with Fried
// parameter r0, kind 1 the step spectrum (tau per FFT cell, i.e. density
// tau L^2, inside the band: |m|^2 <= 9^p band_q2 for the level-p mode
// f = m / (3^p L), band_q2 = (kappa_h L / 2 pi)^2 (1 + 2^-40)).
struct SubharmonicSpec {
  int32_t levels;
  int32_t kind;
  double r0;
  double tau;
  double band_q2;
  double length;
};

// One beam with subharmonics: its axis table (levels x n complex, FP64) at
// tab_off and its pairs' coefficient blocks at coef_off (doubles into the
// subharmonic region of the workspace).
struct SubBeam {
  int32_t inst;
  int32_t n;
  int32_t pairs;
  uint32_t k0, k1;  // Philox key (the beam's seed)
  int32_t pad;
  SubharmonicSpec sp;
  int64_t tab_off;
  int64_t coef_off;
};

// Doubles of a beam's region: tables for the maximum level count and one
// coefficient block per pair.
inline int64_t subharmonic_region_doubles(int n, int pairs) {
  return 2 * int64_t(kMaxSubharmonicLevels) * n + int64_t(kSubPair) * pairs;
}

// Coefficients, means and axis tables of every listed beam and pair (two
// launches).  max_pairs, max_table: the largest pair count and levels x n.
hipError_t launch_subharmonic_setup(const SubBeam* beams, int n_beams, int max_pairs,
                                    int64_t max_table, double* region, hipStream_t s);
// Adds pair `pair`'s low-frequency part to the screen planes of every listed
// beam that has that pair (one launch).  max_n2: the largest n^2.
template <typename R>
hipError_t launch_subharmonic_apply(const SubBeam* beams, int n_beams, const InstDev* inst,
                                    int pair, int64_t max_n2, const double* region, void* planes,
                                    hipStream_t s);

}  // namespace ssfm

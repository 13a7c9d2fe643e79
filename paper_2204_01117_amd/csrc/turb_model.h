// k-omega model constants (Table 1 of the paper), shared by the turbulence
// update and its reverse.
#pragma once

namespace uf {

constexpr double kCmu = 0.09, kAlpha = 0.52, kBeta = 0.0708, kSigma = 0.5, kSigmaStar = 0.6;

}  // namespace uf

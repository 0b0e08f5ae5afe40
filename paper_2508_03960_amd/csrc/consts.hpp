// Physical constants of the simulator (host and device).
#pragma once

namespace gbs {

// gamma/2pi of the proton, Hz/T (CODATA 2018).
constexpr double kGammaBar = 42.577478518e6;
constexpr double kTwoPi = 6.283185307179586476925286766559005768;
constexpr double kPi = 3.141592653589793238462643383279502884;

}  // namespace gbs

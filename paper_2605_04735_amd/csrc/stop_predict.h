// Host-side guess of when an iterative loop will stop (plain C++, no HIP, so
// that the host test suite can compile it on its own).
//
// The loops that run on the device in chunks (the inner CG, the extension CG,
// reinitialisation) stop themselves, and a launch after the stop returns at
// once; the host only chooses how many launches to queue before it looks at
// the state again.  It assumes the watched quantity (a squared residual, the
// largest change of a step) keeps decaying at its mean rate between the last
// two looks, and queues about as many steps as that predicts.
#pragma once

#include <cmath>
#include <limits>

namespace topo {

// Steps after step s1 until a quantity seen as q0 after step s0 and q1 after
// step s1 falls to `target`, at the mean geometric decay rate between the two
// looks.  Zero or negative when q1 is already at or below the target; +inf
// when the inputs give no decay to extrapolate (q did not fall, s1 <= s0, or
// a value is not finite and positive).
inline double predicted_steps(double q0, double s0, double q1, double s1, double target) {
  const double inf = std::numeric_limits<double>::infinity();
  if (!(s1 > s0) || !(q0 > 0.0) || !(q1 > 0.0) || !(target > 0.0) || !std::isfinite(q0) ||
      !std::isfinite(q1) || !std::isfinite(target) || !(q1 < q0))
    return inf;
  const double rate = std::log(q1 / q0) / (s1 - s0);  // < 0
  return std::log(target / q1) / rate;
}

}  // namespace topo

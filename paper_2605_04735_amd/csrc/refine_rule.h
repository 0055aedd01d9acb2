// Stopping rule of the float64 iterative refinement (plain C++, no HIP, so
// that the host test suite can compile it on its own).
//
// The refinement reaches its attainable accuracy when rounding in the float64
// residual r = f - K u, not the inner solve, limits progress.  The rule: stop
// once four consecutive refinement passes have failed to halve the float64
// relative residual, i.e. the residual after pass n exceeds half the residual
// after pass n - 4.  One StagnationRule serves one solve; record() takes the
// residual before the first pass and after every pass, in order.
#pragma once

namespace topo {

struct StagnationRule {
  double hist[4] = {0.0, 0.0, 0.0, 0.0};  // the last four residuals recorded
  int n = 0;                              // residuals recorded so far

  // Records `rel`; true when it is not below half the residual recorded four
  // records earlier.  The slot read is the one about to be overwritten.
  bool record(double rel) {
    const bool stalled = n >= 4 && !(rel <= 0.5 * hist[n % 4]);
    hist[n % 4] = rel;
    ++n;
    return stalled;
  }
};

}  // namespace topo

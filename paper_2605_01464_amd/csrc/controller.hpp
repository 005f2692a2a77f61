// Stop-rule controller: a pure function of per-update scalars (no GPU use).
//
// Rules (the stopping test of Algorithms 1-3 and its variants):
//   DX_ABS   ||X_{j+1} - X_j||_F < tol
//   DX_REL   ||X_{j+1} - X_j||_F <= tol ||X_{j+1}||_F
//   E1_REL   ||A X_{j+1} A - A||_F / ||A||_F <= tol
//   GUARDED  d_j = ||X_{j+1} - X_j||_F / ||X_{j+1}||_F <= tol, or the first rise d_j > d_{j-1} once d
//            has dropped below half of its running maximum.  The update with the smallest d so far
//            is reported as a new minimum so that the driver keeps the two iterates around it.
// An absolute or relative change that is not finite is divergence.
#pragma once

#include <hip/hip_runtime.h>

namespace qp {

#define QP_HD __host__ __device__

enum StopRule : int { STOP_DX_ABS = 0, STOP_DX_REL = 1, STOP_E1_REL = 2, STOP_GUARDED = 3 };
enum Decision : int { D_CONTINUE = 0, D_TOL = 1, D_RISE = 2, D_DIVERGED = 3, D_NEWMIN = 4 };

struct StopController {
  int rule;
  double tol;
  double dmax = 0.0;
  double dprev = -1.0;
  double best_d = __builtin_huge_val();
  int best_j = -1;

  QP_HD StopController() : rule(STOP_GUARDED), tol(0.0) {}
  QP_HD StopController(int r, double t) : rule(r), tol(t) {}

  // j = index of the new iterate X_j (1-based update count).
  QP_HD __attribute__((always_inline)) int update(int j, double d_abs, double x_norm, double e1_rel) {
    if (!__builtin_isfinite(d_abs) || !__builtin_isfinite(x_norm)) return D_DIVERGED;
    switch (rule) {
      case STOP_DX_ABS:
        return d_abs < tol ? D_TOL : D_CONTINUE;
      case STOP_DX_REL:
        return d_abs <= tol * x_norm ? D_TOL : D_CONTINUE;
      case STOP_E1_REL:
        if (!__builtin_isfinite(e1_rel)) return D_DIVERGED;
        return e1_rel <= tol ? D_TOL : D_CONTINUE;
      default: {
        const double d = x_norm > 0.0 ? d_abs / x_norm : 0.0;
        if (d <= tol) return D_TOL;
        int res = D_CONTINUE;
        if (d < best_d) {
          best_d = d;
          best_j = j;
          res = D_NEWMIN;
        }
        if (dprev >= 0.0 && d > dprev && dprev < 0.5 * dmax) return D_RISE;
        if (d > dmax) dmax = d;
        dprev = d;
        return res;
      }
    }
  }
};

}  // namespace qp

// Global quaternion Krylov solvers for A X = B (the Gl-QFOM / Gl-QGMRES of the paper's preconditioning
// experiment), optionally left-preconditioned by an approximate inverse M: M A X = M B.
#pragma once

#include "solver.hpp"

namespace qp {

struct KrylovResult {
  int iters = 0;          // Arnoldi steps taken
  double rr = 0.0;        // relative residual of the iterated system at the last step
  double true_rr = 0.0;   // ||B - A X||_F / ||B - A X_0||_F of the returned X
  int status = QPINV_OK;  // QPINV_ENOTCONVERGED when max_iter steps did not reach tol
};

// method 0: FOM (H_k y = beta e_1), 1: GMRES (min ||beta e_1 - Hbar_k y||).  FP64 matrices; X holds X_0 on
// entry and the solution on return.  history (host, may be null) receives rr after every step.
KrylovResult gl_krylov(Ctx& c, int method, const Mat& A, const Mat& B, const Mat* M, const Mat& X, double tol,
                       int max_iter, double* history, int history_cap, hipStream_t s);

}  // namespace qp

// Memory-bound helper kernels of the solve (host interface).
#pragma once

#include "common.hpp"

namespace qp {

// X = alpha A^H for an m x n quaternion A: X_p[j][i] = alpha * sign_p * A_p[i][j], sign = (+,-,-,-).
// Tin/Tout in {float, double} (the conversion is fused).
template <class Tin, class Tout>
void x0_scaled_adjoint(const QView& A, int64_t m, int64_t n, double alpha, const QView& X, hipStream_t s);

// Y = X elementwise (with type conversion), rows x cols.
template <class Tin, class Tout>
void convert(const QView& X, const QView& Y, int64_t rows, int64_t cols, hipStream_t s);

// Scaling features of A (m x n) written to out[0..3] (device doubles):
//   out[0] = ||A||_F^2, out[1] = ||A||_1 (max column sum of moduli), out[2] = ||A||_inf (max row sum),
//   out[3] = number of non-finite components.
// `work` must hold norms_work_doubles(m, n) doubles.
template <class T>
void norms(const QView& A, int64_t m, int64_t n, double* out, double* work, hipStream_t s);

// Power iteration on A^H A (k steps) from the SplitMix64 start vector; writes the last Rayleigh
// quotient ||A v||^2 (v unit) to lambda[0] and the one of the step before to lambda[1] (device
// doubles; equal when steps == 1).  `work` must hold power_work_doubles(m, n) doubles.
template <class T>
void power_sigma1_sq(const QView& A, int64_t m, int64_t n, int steps, uint64_t seed, double* lambda,
                     double* work, hipStream_t s);
int64_t power_work_doubles(int64_t m, int64_t n);
int64_t norms_work_doubles(int64_t m, int64_t n);

// out[0] = sum |M - M^H|^2 and out[1] = sum |M|^2 over a square quaternion matrix of order n.
// `work` must hold 2 * hermdiff_blocks(n) doubles.
template <class T>
void herm_diff(const QView& M, int64_t n, double* out, double* work, hipStream_t s);
int64_t hermdiff_blocks(int64_t n);

// Xn = Xc + D (FP64 iterates, FP32 correction D), rows x cols, and the change norms
// out[0] = sum |Xn - Xc|^2, out[1] = sum |Xn|^2 (device doubles, fixed summation order).
// `work` must hold 2 * add_delta_blocks(rows, cols) doubles.
void add_delta(const QView& Xc, const QView& D, const QView& Xn, int64_t rows, int64_t cols, double* out,
               double* work, hipStream_t s);
int64_t add_delta_blocks(int64_t rows, int64_t cols);

// Write `count` zeros to device doubles (a kernel, so it is safe inside captured graphs).
void zero_doubles(double* p, int64_t count, hipStream_t s);
template <class T>
void fill_pattern(T* p, int64_t count, hipStream_t s);  // deterministic values in [-1, 1)

}  // namespace qp

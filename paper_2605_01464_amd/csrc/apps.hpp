// Elementwise kernels of the application workloads around the pseudoinverse (Section 5.1's CUR
// completion): submatrix selection by index sets and the masked merge of the impute step.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace qp {

// B = A[rows, cols] for all four planes; rows / cols are DEVICE index arrays (nullptr: all, in
// order).  An index outside A gives a NaN element (the read address is clamped into A).
template <class T>
void submatrix(const QView& A, int64_t m, int64_t n, const int* rows, int64_t nr, const int* cols, int64_t nc,
               const QView& B, hipStream_t s);

// Y = mask ? M : X elementwise for all four planes (mask: DEVICE bytes, rows x cols, row stride mask_ld).
template <class T>
void masked_merge(const QView& M, const unsigned char* mask, int64_t mask_ld, const QView& X, const QView& Y,
                  int64_t rows, int64_t cols, hipStream_t s);

}  // namespace qp

// Elementwise kernels of the application workloads (Section 5.1's CUR completion).  Both are pure
// data movement: coalesced along rows, one plane per grid z-slice.
#include <cmath>
#include <limits>

#include "apps.hpp"

namespace qp {

template <class T>
__global__ void __launch_bounds__(256) submatrix_kernel(const T* __restrict__ A, int64_t lda, int64_t psa, int m, int n,
                                                        const int* __restrict__ rows, int nr, const int* __restrict__ cols,
                                                        int nc, T* __restrict__ B, int64_t ldb, int64_t psb) {
  const int p = blockIdx.z;
  const int64_t total = (int64_t)nr * nc;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / nc), j = (int)(e - (int64_t)i * nc);
    const int ri = rows ? rows[i] : i, cj = cols ? cols[j] : j;
    const bool ok = ri >= 0 && ri < m && cj >= 0 && cj < n;
    const int64_t src = (int64_t)(ok ? ri : 0) * lda + (ok ? cj : 0);
    const T v = A[p * psa + src];
    B[p * psb + (int64_t)i * ldb + j] = ok ? v : std::numeric_limits<T>::quiet_NaN();
  }
}

template <class T>
void submatrix(const QView& A, int64_t m, int64_t n, const int* rows, int64_t nr, const int* cols, int64_t nc,
               const QView& B, hipStream_t s) {
  if (nr == 0 || nc == 0) return;
  const int64_t total = nr * nc;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(submatrix_kernel<T>, dim3(blocks, 1, 4), dim3(256), 0, s, static_cast<const T*>(A.p), A.ld, A.ps,
                     (int)m, (int)n, rows, (int)nr, cols, (int)nc, static_cast<T*>(B.p), B.ld, B.ps);
  QP_HIP(hipGetLastError());
}

template <class T>
__global__ void __launch_bounds__(256) masked_merge_kernel(const T* M, int64_t ldm, int64_t psm,
                                                           const unsigned char* __restrict__ mask, int64_t mask_ld,
                                                           const T* X, int64_t ldx, int64_t psx, T* Y,
                                                           int64_t ldy, int64_t psy, int rows, int cols) {
  const int p = blockIdx.z;
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e - i * cols;
    const T v = mask[i * mask_ld + j] ? M[p * psm + i * ldm + j] : X[p * psx + i * ldx + j];
    Y[p * psy + i * ldy + j] = v;
  }
}

template <class T>
void masked_merge(const QView& M, const unsigned char* mask, int64_t mask_ld, const QView& X, const QView& Y,
                  int64_t rows, int64_t cols, hipStream_t s) {
  if (rows == 0 || cols == 0) return;
  const int64_t total = rows * cols;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(masked_merge_kernel<T>, dim3(blocks, 1, 4), dim3(256), 0, s, static_cast<const T*>(M.p), M.ld,
                     M.ps, mask, mask_ld, static_cast<const T*>(X.p), X.ld, X.ps, static_cast<T*>(Y.p), Y.ld, Y.ps,
                     (int)rows, (int)cols);
  QP_HIP(hipGetLastError());
}

template void submatrix<float>(const QView&, int64_t, int64_t, const int*, int64_t, const int*, int64_t, const QView&,
                               hipStream_t);
template void submatrix<double>(const QView&, int64_t, int64_t, const int*, int64_t, const int*, int64_t, const QView&,
                                hipStream_t);
template void masked_merge<float>(const QView&, const unsigned char*, int64_t, const QView&, const QView&, int64_t,
                                  int64_t, hipStream_t);
template void masked_merge<double>(const QView&, const unsigned char*, int64_t, const QView&, const QView&, int64_t,
                                   int64_t, hipStream_t);

}  // namespace qp

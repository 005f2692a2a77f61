// Memory-bound kernels around the GEMM chain: the initial iterate X_0 = alpha A^H, precision
// conversions, norms and finiteness, the power iteration that estimates sigma_1^2, and the
// Hermitian-difference norms of the Penrose residuals (c), (d).
#include <algorithm>
#include <cmath>

#include "aux.hpp"
#include "qgemm.hpp"

namespace qp {

// ------------------------------------------------------------------------------------------------
// X = alpha A^H  (tiled transpose through LDS; the imaginary planes change sign)
// ------------------------------------------------------------------------------------------------
template <class Tin, class Tout>
__global__ void __launch_bounds__(256) x0_kernel(const Tin* __restrict__ A, int64_t lda, int64_t psa, Tout* __restrict__ X,
                                                 int64_t ldx, int64_t psx, int m, int n, double alpha) {
  __shared__ Tin tile[32][33];
  const int p = blockIdx.z;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const Tin* Ap = A + p * psa;
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    tile[r][tx] = (i < m && j < n) ? Ap[(int64_t)i * lda + j] : Tin(0);
  }
  __syncthreads();
  const double sc = (p == 0) ? alpha : -alpha;
  Tout* Xp = X + p * psx;
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + r, i = i0 + tx;
    if (j < n && i < m) Xp[(int64_t)j * ldx + i] = (Tout)(sc * (double)tile[tx][r]);
  }
}

template <class Tin, class Tout>
void x0_scaled_adjoint(const QView& A, int64_t m, int64_t n, double alpha, const QView& X, hipStream_t s) {
  if (m == 0 || n == 0) return;
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32), 4);
  hipLaunchKernelGGL((x0_kernel<Tin, Tout>), grid, dim3(256), 0, s, static_cast<const Tin*>(A.p), A.ld, A.ps,
                     static_cast<Tout*>(X.p), X.ld, X.ps, (int)m, (int)n, alpha);
  QP_HIP(hipGetLastError());
}

template void x0_scaled_adjoint<float, float>(const QView&, int64_t, int64_t, double, const QView&, hipStream_t);
template void x0_scaled_adjoint<double, double>(const QView&, int64_t, int64_t, double, const QView&, hipStream_t);
template void x0_scaled_adjoint<float, double>(const QView&, int64_t, int64_t, double, const QView&, hipStream_t);
template void x0_scaled_adjoint<double, float>(const QView&, int64_t, int64_t, double, const QView&, hipStream_t);

// ------------------------------------------------------------------------------------------------
// conversion / copy
// ------------------------------------------------------------------------------------------------
template <class Tin, class Tout>
__global__ void __launch_bounds__(256) convert_kernel(const Tin* __restrict__ X, int64_t ldx, int64_t psx, Tout* __restrict__ Y,
                                                      int64_t ldy, int64_t psy, int rows, int cols) {
  const int p = blockIdx.z;
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e - i * cols;
    Y[p * psy + i * ldy + j] = (Tout)X[p * psx + i * ldx + j];
  }
}

template <class Tin, class Tout>
void convert(const QView& X, const QView& Y, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows == 0 || cols == 0) return;
  const int64_t total = rows * cols;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL((convert_kernel<Tin, Tout>), dim3(blocks, 1, 4), dim3(256), 0, s, static_cast<const Tin*>(X.p), X.ld,
                     X.ps, static_cast<Tout*>(Y.p), Y.ld, Y.ps, (int)rows, (int)cols);
  QP_HIP(hipGetLastError());
}

template void convert<float, float>(const QView&, const QView&, int64_t, int64_t, hipStream_t);
template void convert<double, double>(const QView&, const QView&, int64_t, int64_t, hipStream_t);
template void convert<float, double>(const QView&, const QView&, int64_t, int64_t, hipStream_t);
template void convert<double, float>(const QView&, const QView&, int64_t, int64_t, hipStream_t);

// ------------------------------------------------------------------------------------------------
// small reductions (single workgroup, fixed order)
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256) zero_kernel(double* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = 0.0;
}

void zero_doubles(double* p, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, p, count);
  QP_HIP(hipGetLastError());
}

__global__ void __launch_bounds__(256) add_delta_kernel(const double* __restrict__ Xc, int64_t ldc, int64_t psc,
                                                        const float* __restrict__ D, int64_t ldd, int64_t psd,
                                                        double* __restrict__ Xn, int64_t ldn, int64_t psn, int rows,
                                                        int cols, double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t total = (int64_t)rows * cols;
  double sd = 0.0, sx = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e - i * cols;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const double xc = Xc[p * psc + i * ldc + j];
      const double xn = xc + (double)D[p * psd + i * ldd + j];
      Xn[p * psn + i * ldn + j] = xn;
      const double dd = xn - xc;
      sd += dd * dd;
      sx += xn * xn;
    }
  }
  const double a = block_sum256(sd, sh);
  const double b = block_sum256(sx, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

int64_t add_delta_blocks(int64_t rows, int64_t cols) {
  return std::max<int64_t>(1, std::min<int64_t>((rows * cols + 255) / 256, 1024));
}

void add_delta(const QView& Xc, const QView& D, const QView& Xn, int64_t rows, int64_t cols, double* out,
               double* work, hipStream_t s) {
  const int64_t nb = add_delta_blocks(rows, cols);
  hipLaunchKernelGGL(add_delta_kernel, dim3((unsigned)nb), dim3(256), 0, s, static_cast<const double*>(Xc.p), Xc.ld,
                     Xc.ps, static_cast<const float*>(D.p), D.ld, D.ps, static_cast<double*>(Xn.p), Xn.ld, Xn.ps,
                     (int)rows, (int)cols, work);
  QP_HIP(hipGetLastError());
  reduce_pairs(work, nb, out, s);
}

// Values in [-1, 1) from a multiplicative hash of the index (timing inputs: MFMA power and thus clocks
// depend on the operand bits, so tiles are timed on dense data rather than zeros).
template <class T>
__global__ void __launch_bounds__(256) fill_kernel(T* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
    const uint32_t h = (uint32_t)(i * 2654435761ull) ^ (uint32_t)(i >> 17);
    p[i] = (T)((double)(h >> 8) * 0x1p-23 - 1.0);
  }
}

template <class T>
void fill_pattern(T* p, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks), dim3(256), 0, s, p, count);
  QP_HIP(hipGetLastError());
}
template void fill_pattern<float>(float*, int64_t, hipStream_t);
template void fill_pattern<double>(double*, int64_t, hipStream_t);

// ------------------------------------------------------------------------------------------------
// norms: row pass (one workgroup per row), column pass (column strips x row blocks), finalize
// ------------------------------------------------------------------------------------------------
static int col_row_blocks(int64_t m) { return (int)std::max<int64_t>(1, std::min<int64_t>(64, (m + 63) / 64)); }

template <class T>
__global__ void __launch_bounds__(256) norms_row_kernel(const T* __restrict__ A, int64_t lda, int64_t psa, int n,
                                                        double* __restrict__ row_abs, double* __restrict__ row_sq,
                                                        double* __restrict__ row_nf) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  double sa = 0.0, sq = 0.0, nf = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    double q2 = 0.0;
    for (int p = 0; p < 4; ++p) {
      const double v = (double)A[p * psa + (int64_t)i * lda + j];
      if (!isfinite(v)) nf += 1.0;
      q2 += v * v;
    }
    sq += q2;
    sa += sqrt(q2);
  }
  sa = block_sum256(sa, sh);
  sq = block_sum256(sq, sh);
  nf = block_sum256(nf, sh);
  if (threadIdx.x == 0) {
    row_abs[i] = sa;
    row_sq[i] = sq;
    row_nf[i] = nf;
  }
}

template <class T>
__global__ void __launch_bounds__(256) norms_col_kernel(const T* __restrict__ A, int64_t lda, int64_t psa, int m, int n,
                                                        double* __restrict__ col_part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int rb = blockIdx.y, nrb = gridDim.y;
  const int per = (m + nrb - 1) / nrb;
  const int r0 = rb * per, r1 = min(m, r0 + per);
  if (j >= n) return;
  double sa = 0.0;
  for (int i = r0; i < r1; ++i) {
    double q2 = 0.0;
    for (int p = 0; p < 4; ++p) {
      const double v = (double)A[p * psa + (int64_t)i * lda + j];
      q2 += v * v;
    }
    sa += sqrt(q2);
  }
  col_part[(int64_t)rb * n + j] = sa;
}

__global__ void __launch_bounds__(256) norms_final_kernel(const double* __restrict__ row_abs, const double* __restrict__ row_sq,
                                                          const double* __restrict__ row_nf, const double* __restrict__ col_part,
                                                          int m, int n, int nrb, double* __restrict__ out) {
  __shared__ double sh[256];
  double fro = 0.0, rmax = 0.0, nf = 0.0, cmax = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    fro += row_sq[i];
    rmax = fmax(rmax, row_abs[i]);
    nf += row_nf[i];
  }
  for (int j = threadIdx.x; j < n; j += 256) {
    double c = 0.0;
    for (int rb = 0; rb < nrb; ++rb) c += col_part[(int64_t)rb * n + j];
    cmax = fmax(cmax, c);
  }
  fro = block_sum256(fro, sh);
  nf = block_sum256(nf, sh);
  rmax = block_max256(rmax, sh);
  cmax = block_max256(cmax, sh);
  if (threadIdx.x == 0) {
    out[0] = fro;
    out[1] = cmax;
    out[2] = rmax;
    out[3] = nf;
  }
}

int64_t norms_work_doubles(int64_t m, int64_t n) { return 3 * m + (int64_t)col_row_blocks(m) * n + 8; }

template <class T>
void norms(const QView& A, int64_t m, int64_t n, double* out, double* work, hipStream_t s) {
  if (m == 0 || n == 0) {
    zero_doubles(out, 4, s);
    return;
  }
  double* row_abs = work;
  double* row_sq = work + m;
  double* row_nf = work + 2 * m;
  double* col_part = work + 3 * m;
  const int nrb = col_row_blocks(m);
  hipLaunchKernelGGL((norms_row_kernel<T>), dim3((unsigned)m), dim3(256), 0, s, static_cast<const T*>(A.p), A.ld, A.ps,
                     (int)n, row_abs, row_sq, row_nf);
  QP_HIP(hipGetLastError());
  hipLaunchKernelGGL((norms_col_kernel<T>), dim3((unsigned)((n + 255) / 256), (unsigned)nrb), dim3(256), 0, s,
                     static_cast<const T*>(A.p), A.ld, A.ps, (int)m, (int)n, col_part);
  QP_HIP(hipGetLastError());
  hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(256), 0, s, row_abs, row_sq, row_nf, col_part, (int)m, (int)n, nrb,
                     out);
  QP_HIP(hipGetLastError());
}

template void norms<float>(const QView&, int64_t, int64_t, double*, double*, hipStream_t);
template void norms<double>(const QView&, int64_t, int64_t, double*, double*, hipStream_t);

// ------------------------------------------------------------------------------------------------
// power iteration on A^H A
//   v_0[p][j] = u(splitmix64(p n + j)), u(z) = (z >> 11) 2^-52 - 1;
//   repeat: v <- v / ||v||; w = A v; lambda = ||w||^2; v <- A^H w.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t counter, uint64_t seed) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) power_init_kernel(double* v, int n, uint64_t seed) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < 4 * n) v[e] = (double)(splitmix64((uint64_t)e, seed) >> 11) * 0x1p-52 - 1.0;
}

// out[0] = sum of squares of x[0..len); if prev != nullptr the old out[0] is moved to prev[0] first
__global__ void __launch_bounds__(256) sumsq_kernel(const double* __restrict__ x, int64_t len, double* __restrict__ out,
                                                    double* __restrict__ prev) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += 256) a += x[i] * x[i];
  a = block_sum256(a, sh);
  if (threadIdx.x == 0) {
    if (prev) prev[0] = out[0];
    out[0] = a;
  }
}

// w_i = (A v)_i / sqrt(*vn2): one workgroup per row.  v and w are plane-major (4 x len).
template <class T>
__global__ void __launch_bounds__(256) gemv_n_kernel(const T* __restrict__ A, int64_t lda, int64_t psa, int m, int n,
                                                     const double* __restrict__ v, const double* __restrict__ vn2,
                                                     double* __restrict__ w) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const int64_t o = (int64_t)i * lda + j;
    const double as = A[o], ax = A[psa + o], ay = A[2 * psa + o], az = A[3 * psa + o];
    const double vs = v[j], vx = v[n + j], vy = v[2 * n + j], vz = v[3 * n + j];
    s0 += as * vs - ax * vx - ay * vy - az * vz;
    s1 += as * vx + ax * vs + ay * vz - az * vy;
    s2 += as * vy - ax * vz + ay * vs + az * vx;
    s3 += as * vz + ax * vy - ay * vx + az * vs;
  }
  s0 = block_sum256(s0, sh);
  s1 = block_sum256(s1, sh);
  s2 = block_sum256(s2, sh);
  s3 = block_sum256(s3, sh);
  if (threadIdx.x == 0) {
    const double inv = 1.0 / sqrt(vn2[0]);
    w[i] = s0 * inv;
    w[m + i] = s1 * inv;
    w[2 * m + i] = s2 * inv;
    w[3 * m + i] = s3 * inv;
  }
}

// partial z_j = sum_{i in row block} conj(a_ij) w_i
template <class T>
__global__ void __launch_bounds__(256) gemv_h_kernel(const T* __restrict__ A, int64_t lda, int64_t psa, int m, int n,
                                                     const double* __restrict__ w, double* __restrict__ zpart) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int rb = blockIdx.y, nrb = gridDim.y;
  const int per = (m + nrb - 1) / nrb;
  const int r0 = rb * per, r1 = min(m, r0 + per);
  if (j >= n) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int i = r0; i < r1; ++i) {
    const int64_t o = (int64_t)i * lda + j;
    const double as = A[o], ax = A[psa + o], ay = A[2 * psa + o], az = A[3 * psa + o];
    const double ws = w[i], wx = w[m + i], wy = w[2 * m + i], wz = w[3 * m + i];
    s0 += as * ws + ax * wx + ay * wy + az * wz;
    s1 += as * wx - ax * ws - ay * wz + az * wy;
    s2 += as * wy + ax * wz - ay * ws - az * wx;
    s3 += as * wz - ax * wy + ay * wx - az * ws;
  }
  double* zp = zpart + (int64_t)rb * 4 * n;
  zp[j] = s0;
  zp[n + j] = s1;
  zp[2 * n + j] = s2;
  zp[3 * n + j] = s3;
}

__global__ void __launch_bounds__(256) sum_parts_kernel(const double* __restrict__ part, int nrb, int64_t len,
                                                        double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= len) return;
  double a = 0.0;
  for (int rb = 0; rb < nrb; ++rb) a += part[(int64_t)rb * len + e];
  out[e] = a;
}

__global__ void copy1_kernel(const double* src, double* dst) {
  if (threadIdx.x == 0) dst[0] = src[0];
}

int64_t power_work_doubles(int64_t m, int64_t n) { return 4 * n + 4 * m + (int64_t)col_row_blocks(m) * 4 * n + 8; }

template <class T>
void power_sigma1_sq(const QView& A, int64_t m, int64_t n, int steps, uint64_t seed, double* lambda, double* work,
                     hipStream_t s) {
  if (m == 0 || n == 0 || steps < 1) {
    zero_doubles(lambda, 2, s);
    return;
  }
  double* v = work;
  double* w = v + 4 * n;
  double* zpart = w + 4 * m;
  const int nrb = col_row_blocks(m);
  double* vn2 = zpart + (int64_t)nrb * 4 * n;
  const T* Ap = static_cast<const T*>(A.p);
  hipLaunchKernelGGL(power_init_kernel, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, s, v, (int)n, (uint64_t)seed);
  QP_HIP(hipGetLastError());
  for (int k = 0; k < steps; ++k) {
    hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(256), 0, s, v, 4 * n, vn2, (double*)nullptr);
    hipLaunchKernelGGL((gemv_n_kernel<T>), dim3((unsigned)m), dim3(256), 0, s, Ap, A.ld, A.ps, (int)m, (int)n, v, vn2, w);
    hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(256), 0, s, w, 4 * m, lambda, k > 0 ? lambda + 1 : (double*)nullptr);
    hipLaunchKernelGGL((gemv_h_kernel<T>), dim3((unsigned)((n + 255) / 256), (unsigned)nrb), dim3(256), 0, s, Ap, A.ld,
                       A.ps, (int)m, (int)n, w, zpart);
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, s, zpart, nrb, 4 * n, v);
    QP_HIP(hipGetLastError());
  }
  if (steps == 1) hipLaunchKernelGGL(copy1_kernel, dim3(1), dim3(64), 0, s, lambda, lambda + 1);
}

template void power_sigma1_sq<float>(const QView&, int64_t, int64_t, int, uint64_t, double*, double*, hipStream_t);
template void power_sigma1_sq<double>(const QView&, int64_t, int64_t, int, uint64_t, double*, double*, hipStream_t);

// ------------------------------------------------------------------------------------------------
// Hermitian difference: sum |M_ij - conj(M_ji)|^2 and sum |M_ij|^2
// ------------------------------------------------------------------------------------------------
int64_t hermdiff_blocks(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(1024, (n * n + 255) / 256)); }

template <class T>
__global__ void __launch_bounds__(256) herm_kernel(const T* __restrict__ M, int64_t ld, int64_t ps, int n,
                                                   double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t total = (int64_t)n * n;
  double d = 0.0, x = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, j = e - i * n;
    for (int p = 0; p < 4; ++p) {
      const double a = (double)M[p * ps + i * ld + j];
      const double b = (double)M[p * ps + j * ld + i];
      const double t = (p == 0) ? a - b : a + b;
      d += t * t;
      x += a * a;
    }
  }
  d = block_sum256(d, sh);
  x = block_sum256(x, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = d;
    part[2 * blockIdx.x + 1] = x;
  }
}

template <class T>
void herm_diff(const QView& M, int64_t n, double* out, double* work, hipStream_t s) {
  const int64_t nb = hermdiff_blocks(n);
  if (n == 0) {
    zero_doubles(out, 2, s);
    return;
  }
  hipLaunchKernelGGL((herm_kernel<T>), dim3((unsigned)nb), dim3(256), 0, s, static_cast<const T*>(M.p), M.ld, M.ps, (int)n,
                     work);
  QP_HIP(hipGetLastError());
  reduce_pairs(work, nb, out, s);
}

template void herm_diff<float>(const QView&, int64_t, double*, double*, hipStream_t);
template void herm_diff<double>(const QView&, int64_t, double*, double*, hipStream_t);

}  // namespace qp

// Global quaternion FOM / GMRES.  The Krylov basis V_0, V_1, ... of n x m quaternion matrices is
// orthonormal in <X, Y> = Re tr(X^H Y), which is the real dot product of the four stacked planes, so
// every basis operation is a dense real vector operation over L = 4 n m doubles: the basis lives in one
// device array [k][4][n][m] (each V_j also a quaternion-matrix view for the products), the projections
// are one dot kernel over all previous V_i and one fused multi-axpy (classical Gram-Schmidt, applied
// twice), and only the small Hessenberg matrix and its Givens rotations are handled on the host.
#include <cmath>
#include <vector>

#include "krylov.hpp"

namespace qp {

namespace {

// out[i] = <V_i, W> for i < nvec (one workgroup per i, fixed-order reduction)
__global__ void __launch_bounds__(256) dots_kernel(const double* __restrict__ V, int64_t L, const double* __restrict__ W,
                                                   int nvec, double* __restrict__ out) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  if (i >= nvec) return;
  const double* v = V + (int64_t)i * L;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < L; e += 256) acc += v[e] * W[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// W[e] += sign * sum_i h[i] V_i[e]   (i < nvec, in index order)
__global__ void __launch_bounds__(256) multi_axpy_kernel(const double* __restrict__ V, int64_t L,
                                                         const double* __restrict__ h, int nvec, double sign,
                                                         double* __restrict__ W) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < L; e += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int i = 0; i < nvec; ++i) acc += h[i] * V[(int64_t)i * L + e];
    W[e] += sign * acc;
  }
}

// Y = a X
__global__ void __launch_bounds__(256) scale_kernel(const double* __restrict__ X, int64_t L, double a,
                                                    double* __restrict__ Y) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < L; e += (int64_t)gridDim.x * 256) Y[e] = a * X[e];
}

unsigned blocks_for(int64_t L) { return (unsigned)std::min<int64_t>((L + 255) / 256, 2048); }

// a dense n x m view of slot j of the basis array
Mat slot(double* base, int64_t j, int64_t n, int64_t m) {
  Mat v;
  v.v.p = base + j * 4 * n * m;
  v.v.rows = n;
  v.v.cols = m;
  v.v.ld = m;
  v.v.ps = n * m;
  v.rows = n;
  v.cols = m;
  v.dtype = QPINV_F64;
  return v;
}

// C = A B + beta * In (FP64 product)
void product(Ctx& c, const Mat& A, const Mat& B, const Mat& C, hipStream_t s, const Mat* In = nullptr,
             double a = 1.0, double beta = 0.0) {
  Epilogue e;
  e.nout = 1;
  e.out[0] = C.v;
  e.a[0] = a;
  if (In) {
    e.nin = 1;
    e.in[0] = In->v;
    e.b[0][0] = beta;
  }
  gemm(c, P_F64, A, B, e, s);
}

}  // namespace

KrylovResult gl_krylov(Ctx& c, int method, const Mat& A, const Mat& B, const Mat* M, const Mat& X, double tol,
                       int max_iter, double* history, int history_cap, hipStream_t s) {
  const int64_t n = A.rows, m = B.cols, L = 4 * n * m;
  KrylovResult res;
  // device work: basis (max_iter + 1 slots), the product temporaries, residual, projections
  double* V = static_cast<double*>(c.ws.get("krylov_basis", sizeof(double) * (size_t)(L * (max_iter + 1))));
  double* T = static_cast<double*>(c.ws.get("krylov_tmp", sizeof(double) * (size_t)(4 * L)));
  double* dh = static_cast<double*>(c.ws.get("krylov_h", sizeof(double) * (size_t)(2 * (max_iter + 2) + 1)));
  const Mat W = slot(T, 0, n, m), AV = slot(T, 1, n, m), R0 = slot(T, 2, n, m), Xt = slot(T, 3, n, m);
  std::vector<double> hh(2 * (max_iter + 2) + 1);
  auto fetch = [&](int count) {
    QP_HIP(hipMemcpyAsync(hh.data(), dh, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    QP_HIP(hipStreamSynchronize(s));
  };
  auto dot_self = [&](const double* x) {
    hipLaunchKernelGGL(dots_kernel, dim3(1), dim3(256), 0, s, x, L, x, 1, dh);
    QP_HIP(hipGetLastError());
    fetch(1);
    return hh[0];
  };

  // R_0 = B - A X_0 and the initial residual of the iterated system Z_0 = M R_0 (or R_0)
  product(c, A, X, R0, s, &B, -1.0, 1.0);
  const double r0 = std::sqrt(dot_self(static_cast<double*>(R0.v.p)));
  const Mat Z0 = M ? W : R0;
  if (M) product(c, *M, R0, W, s);
  const double beta = M ? std::sqrt(dot_self(static_cast<double*>(W.v.p))) : r0;
  if (beta == 0.0) {
    res.true_rr = 0.0;
    return res;
  }
  hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(L)), dim3(256), 0, s, static_cast<const double*>(Z0.v.p), L,
                     1.0 / beta, V);
  QP_HIP(hipGetLastError());

  // Hessenberg columns (host), Givens rotations, rotated right-hand side
  std::vector<std::vector<double>> H;  // H[j] = column j (rotated: R's column), length j + 2
  std::vector<double> cs, sn, g(1, beta);
  int k = 0;
  // coefficients y of X_k = X_0 + sum_i y_i V_i after k steps
  auto coefficients = [&](int kk) {
    std::vector<double> y(kk, 0.0);
    if (method == 1) {  // GMRES: upper-triangular R y = g (the rotated Hessenberg)
      for (int i = kk - 1; i >= 0; --i) {
        double t = g[i];
        for (int l = i + 1; l < kk; ++l) t -= H[l][i] * y[l];
        y[i] = t / H[i][i];
      }
    } else {  // FOM: H_k y = beta e_1.  The first k - 1 rotations bring the square Hessenberg to R with
      // its last diagonal entry taken before the last rotation (c rho), and beta e_1 to g with its last
      // entry taken before the last rotation (g / c).
      const double c_last = cs[kk - 1];
      for (int i = kk - 1; i >= 0; --i) {
        double t = (i == kk - 1) ? g[i] / c_last : g[i];
        for (int l = i + 1; l < kk; ++l) t -= H[l][i] * y[l];
        y[i] = t / ((i == kk - 1) ? c_last * H[i][i] : H[i][i]);
      }
    }
    return y;
  };
  // Xdst = X_0 + sum_i y_i V_i (X holds X_0 until the end)
  auto form = [&](int kk, const Mat& Xdst) {
    const std::vector<double> y = coefficients(kk);
    QP_HIP(hipMemcpyAsync(dh, y.data(), sizeof(double) * kk, hipMemcpyHostToDevice, s));
    if (Xdst.v.p != X.v.p)
      QP_HIP(hipMemcpyAsync(Xdst.v.p, X.v.p, sizeof(double) * (size_t)L, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(blocks_for(L)), dim3(256), 0, s, V, L, dh, kk, 1.0,
                       static_cast<double*>(Xdst.v.p));
    QP_HIP(hipGetLastError());
    QP_HIP(hipStreamSynchronize(s));  // y (host) is read by the copy
  };
  // RR = ||B - A Xs||_F / ||B - A X_0||_F
  auto true_residual = [&](const Mat& Xs) {
    product(c, A, Xs, AV, s, &B, -1.0, 1.0);
    return std::sqrt(dot_self(static_cast<double*>(AV.v.p))) / r0;
  };
  res.status = QPINV_ENOTCONVERGED;
  for (int j = 0; j < max_iter; ++j) {
    const Mat Vj = slot(V, j, n, m);
    // W = A V_j, or M (A V_j)
    if (M) {
      product(c, A, Vj, AV, s);
      product(c, *M, AV, W, s);
    } else {
      product(c, A, Vj, W, s);
    }
    // classical Gram-Schmidt, twice: h = V^T W, W -= V h (on device; h to the host once)
    // (both passes and the norm of the result queue back to back; one host synchronisation per step)
    double* w = static_cast<double*>(W.v.p);
    for (int pass = 0; pass < 2; ++pass) {
      double* hp = dh + pass * (j + 1);
      hipLaunchKernelGGL(dots_kernel, dim3(j + 1), dim3(256), 0, s, V, L, w, j + 1, hp);
      QP_HIP(hipGetLastError());
      hipLaunchKernelGGL(multi_axpy_kernel, dim3(blocks_for(L)), dim3(256), 0, s, V, L, hp, j + 1, -1.0, w);
      QP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(dots_kernel, dim3(1), dim3(256), 0, s, w, L, w, 1, dh + 2 * (j + 1));
    QP_HIP(hipGetLastError());
    fetch(2 * (j + 1) + 1);
    std::vector<double> col(j + 2, 0.0);
    for (int i = 0; i <= j; ++i) col[i] = hh[i] + hh[j + 1 + i];
    const double hn = std::sqrt(hh[2 * (j + 1)]);
    col[j + 1] = hn;
    H.push_back(col);
    // apply the previous rotations to the new column, then zero its subdiagonal entry
    std::vector<double>& hc = H.back();
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
      hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
      hc[i] = t;
    }
    const double rho = std::hypot(hc[j], hc[j + 1]);
    const double cj = rho > 0.0 ? hc[j] / rho : 1.0, sj = rho > 0.0 ? hc[j + 1] / rho : 0.0;
    cs.push_back(cj);
    sn.push_back(sj);
    hc[j] = rho;  // the rotated column: R's column j
    hc[j + 1] = 0.0;
    g.push_back(-sj * g[j]);
    g[j] = cj * g[j];
    k = j + 1;
    // GMRES residual |g_{j+1}|; the FOM residual is larger by 1 / |c_j| (Saad, Prop. 6.9)
    const double res_g = std::fabs(g[j + 1]);
    const double res_k = method == 0 ? (std::fabs(cj) > 0.0 ? res_g / std::fabs(cj) : INFINITY) : res_g;
    res.rr = res_k / beta;
    if (history && j < history_cap) history[j] = res.rr;
    bool stop = hn == 0.0;
    if (res.rr <= tol) {
      // the stopping test is on the original system's residual; with M it is checked from here on
      if (!M) {
        stop = true;
      } else {
        form(k, Xt);
        stop = stop || true_residual(Xt) <= tol;
      }
    }
    if (stop) {
      res.status = QPINV_OK;
      break;
    }
    hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(L)), dim3(256), 0, s, static_cast<const double*>(w), L, 1.0 / hn,
                       V + (int64_t)(j + 1) * L);
    QP_HIP(hipGetLastError());
  }
  res.iters = k;

  form(k, X);
  res.true_rr = true_residual(X);
  return res;
}

}  // namespace qp

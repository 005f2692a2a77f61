// Batched pseudoinverses of many small, uneven quaternion matrices in ONE persistent launch.
//
// Every workgroup is a solver: it takes the next matrix from a device work queue (matrices are
// ordered largest work first, so the long solves start early) and runs the whole method on it --
// scaling by power iteration, X_0 = alpha A^H, the fused product chain of the method through the same
// tile routine as the standalone product kernel, and the guarded stop rule -- then takes the next one.
// Workgroups never wait for each other, so the launch cannot deadlock; every loop is bounded by
// the batch size and max_iter.  The host captures upload + queue reset + launch + download in a
// hipGraph and replays it for later batches of the same shape signature.
//
// Per-workgroup scratch: NBUF quaternion buffers of D x D (D = largest dimension in the batch, ld = D)
// for the chain, the iterates and the saved residuals, plus double vectors for the power iteration.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "batched.hpp"
#include "controller.hpp"
#include "qgemm_kern.hpp"

namespace qp {

namespace {
constexpr int NBUF = 17;  // sq 0..9, X 10..13, Rsave 14..15, E2 out 16
constexpr int BX = 10, BR = 14, BE = 16;

const double kS5 = std::sqrt(5.0);
const double kS93 = std::sqrt(93.0);
const double kRt = std::sqrt(27.0 - 2.0 * kS93);

struct Coef {
  float beta1, beta2, d1, d2, d3, e1, e2, c1, c2;
};

Coef make_coef() {
  Coef c;
  c.beta1 = (float)(0.5 * (1.0 + kS5));
  c.beta2 = (float)(0.5 * (1.0 - kS5));
  c.d1 = (float)(0.25 * (1.0 + kRt));
  c.d2 = (float)(0.25 * (1.0 - kRt));
  c.d3 = (float)((5.0 * kS93 - 93.0) / 496.0);
  c.e1 = (float)((-93.0 - 5.0 * kS93) / 496.0);
  c.e2 = (float)(-0.25 * kS93);
  c.c1 = (float)(3.0 / 8.0);
  c.c2 = (float)(321.0 / 1984.0);
  return c;
}
}  // namespace

struct BParams {
  const BDesc* desc;
  BInfo* info;
  const int* order;
  int count;
  int* queue;
  float* work;  // NBUF * 4 * D * D floats per workgroup
  double* dwork;  // 8 * D + 64 doubles per workgroup
  const double* alpha;  // given alpha per matrix (scaling == given)
  int D;
  int method;
  int stop;
  int max_iter;
  double tol;
  int scaling;
  int power_steps;
  unsigned long long seed;
  Coef k;
};

// A matrix view inside the solver: pointer, strides, shape.
struct DM {
  float* p = nullptr;
  int64_t ld = 0, ps = 0;
  int rows = 0, cols = 0;
};

__device__ __forceinline__ uint64_t bsplitmix64(uint64_t counter, uint64_t seed) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// workgroup sum of a double (every thread gets the result)
__device__ __forceinline__ double wg_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  __syncthreads();
  return t;
}

// epilogue description for the in-workgroup product
struct DEpi {
  int nout = 1;
  DM out[3];
  float a[3] = {1.f, 1.f, 1.f};
  int nin = 0;
  DM in[3];
  float b[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  float g[3] = {0.f, 0.f, 0.f};
  int reduce = 0;
  int ref = -1;
};

__device__ __forceinline__ DEpi epi_out(const DM& o, float a = 1.f, float g = 0.f) {
  DEpi e;
  e.out[0] = o;
  e.a[0] = a;
  e.g[0] = g;
  return e;
}

// C = A B with the epilogue, all tiles of the output walked by this workgroup; returns the
// workgroup totals of the reduction terms in (sd, sx) when e.reduce.
template <class MM, int BM, int BN, int BK, int WM, int WN>
__device__ __attribute__((noinline)) void wg_gemm(const DM& A, const DM& B, const DEpi& e, float* smem, double* sh,
                                                  double& sd, double& sx) {
  GemmParams<float> P;
  P.A = A.p;
  P.lda = A.ld;
  P.psa = A.ps;
  P.B = B.p;
  P.ldb = B.ld;
  P.psb = B.ps;
  P.M = A.rows;
  P.N = B.cols;
  P.K = A.cols;
  P.tiles_m = (P.M + BM - 1) / BM;
  P.tiles_n = (P.N + BN - 1) / BN;
  P.vec = ((A.ld | A.ps | B.ld | B.ps) & 3) == 0;
  P.nout = e.nout;
  P.nin = e.nin;
  P.ref = e.ref;
  for (int t = 0; t < 3; ++t) {
    P.out[t] = e.out[t].p;
    P.ldo[t] = e.out[t].ld;
    P.pso[t] = e.out[t].ps;
    P.in[t] = e.in[t].p;
    P.ldi[t] = e.in[t].ld;
    P.psi[t] = e.in[t].ps;
    P.ca[t] = e.a[t];
    P.cg[t] = e.g[t];
    for (int u = 0; u < 3; ++u) P.cb[t][u] = e.b[t][u];
  }
  P.partial = nullptr;
  P.reduce = e.reduce;
  double a0 = 0.0, a1 = 0.0;
  const int nt = P.tiles_m * P.tiles_n;
  for (int t = 0; t < nt; ++t) gemm_tile<MM, BM, BN, BK, WM, WN, 128>(P, t / P.tiles_n, t % P.tiles_n, smem, a0, a1);
  if (e.reduce) {
    sd = wg_sum(a0, sh);
    sx = wg_sum(a1, sh);
  }
  __threadfence_block();
  __syncthreads();
}

template <class MM, int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) batched_kernel(BParams P) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  __shared__ float smem[C::SMEM];
  __shared__ double sh[16];
  __shared__ int s_next;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int D = P.D;
  const int64_t PS = (int64_t)D * D;
  float* const W = P.work + (int64_t)blockIdx.x * NBUF * 4 * PS;
  double* const dw = P.dwork + (int64_t)blockIdx.x * (8 * (int64_t)D + 64);
  auto buf = [&](int k, int rows, int cols) {
    DM v;
    v.p = W + (int64_t)k * 4 * PS;
    v.ld = D;
    v.ps = PS;
    v.rows = rows;
    v.cols = cols;
    return v;
  };

  for (int guard = 0; guard <= P.count; ++guard) {
    if (tid == 0) s_next = atomicAdd(P.queue, 1);
    __syncthreads();
    const int slot = s_next;
    __syncthreads();
    if (slot >= P.count) break;
    const int b = P.order[slot];
    const BDesc d = P.desc[b];
    const int m = d.m, n = d.n;
    DM A;
    A.p = const_cast<float*>(d.A);
    A.ld = d.lda;
    A.ps = d.psa;
    A.rows = m;
    A.cols = n;
    const bool left = m > n;
    const int s = left ? n : m;
    BInfo info;
    info.iters = 0;
    info.returned = 0;
    info.reason = 0;
    info.status = 0;
    info.alpha = 0.0;
    info.dx_rel = 0.0;
    info.sigma1_sq = 0.0;

    // ---------------------------------------------------------------- norm and finiteness of A
    double fro2 = 0.0, nf = 0.0;
    for (int e = tid; e < m * n; e += nthr) {
      const int i = e / n, j = e - i * n;
      for (int p = 0; p < 4; ++p) {
        const double v = A.p[p * A.ps + (int64_t)i * A.ld + j];
        if (!__builtin_isfinite(v)) nf += 1.0;
        fro2 += v * v;
      }
    }
    fro2 = wg_sum(fro2, sh);
    nf = wg_sum(nf, sh);
    if (nf > 0.0) {
      info.status = -2;
      if (tid == 0) P.info[b] = info;
      continue;
    }
    const double normA = sqrt(fro2);

    // ---------------------------------------------------------------- scaling
    double alpha;
    if (P.scaling == 2) {
      alpha = P.alpha[b];
    } else {
      double* v = dw;          // 4n
      double* wv = dw + 4 * D;  // 4m
      for (int e = tid; e < 4 * n; e += nthr) v[e] = (double)(bsplitmix64((uint64_t)e, P.seed) >> 11) * 0x1p-52 - 1.0;
      __syncthreads();
      double lam = 0.0;
      for (int k = 0; k < P.power_steps; ++k) {
        double nv = 0.0;
        for (int e = tid; e < 4 * n; e += nthr) nv += v[e] * v[e];
        nv = wg_sum(nv, sh);
        const double inv = 1.0 / sqrt(nv);
        for (int i = tid; i < m; i += nthr) {
          double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
          for (int j = 0; j < n; ++j) {
            const int64_t o = (int64_t)i * A.ld + j;
            const double as = A.p[o], ax = A.p[A.ps + o], ay = A.p[2 * A.ps + o], az = A.p[3 * A.ps + o];
            const double vs = v[j], vx = v[n + j], vy = v[2 * n + j], vz = v[3 * n + j];
            s0 += as * vs - ax * vx - ay * vy - az * vz;
            s1 += as * vx + ax * vs + ay * vz - az * vy;
            s2 += as * vy - ax * vz + ay * vs + az * vx;
            s3 += as * vz + ax * vy - ay * vx + az * vs;
          }
          wv[i] = s0 * inv;
          wv[m + i] = s1 * inv;
          wv[2 * m + i] = s2 * inv;
          wv[3 * m + i] = s3 * inv;
        }
        __syncthreads();
        double l2 = 0.0;
        for (int e = tid; e < 4 * m; e += nthr) l2 += wv[e] * wv[e];
        lam = wg_sum(l2, sh);
        for (int j = tid; j < n; j += nthr) {
          double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
          for (int i = 0; i < m; ++i) {
            const int64_t o = (int64_t)i * A.ld + j;
            const double as = A.p[o], ax = A.p[A.ps + o], ay = A.p[2 * A.ps + o], az = A.p[3 * A.ps + o];
            const double ws = wv[i], wx = wv[m + i], wy = wv[2 * m + i], wz = wv[3 * m + i];
            s0 += as * ws + ax * wx + ay * wy + az * wz;
            s1 += as * wx - ax * ws - ay * wz + az * wy;
            s2 += as * wy + ax * wz - ay * ws - az * wx;
            s3 += as * wz - ax * wy + ay * wx - az * ws;
          }
          v[j] = s0;
          v[n + j] = s1;
          v[2 * n + j] = s2;
          v[3 * n + j] = s3;
        }
        __syncthreads();
      }
      info.sigma1_sq = lam;
      alpha = 1.0 / lam;
    }
    info.alpha = alpha;

    // ---------------------------------------------------------------- X_0 = alpha A^H
    DM X[4] = {buf(BX, n, m), buf(BX + 1, n, m), buf(BX + 2, n, m), buf(BX + 3, n, m)};
    for (int e = tid; e < m * n; e += nthr) {
      const int i = e / n, j = e - i * n;
      for (int p = 0; p < 4; ++p)
        X[0].p[p * PS + (int64_t)j * D + i] = (float)((p == 0 ? alpha : -alpha) * (double)A.p[p * A.ps + (int64_t)i * A.ld + j]);
    }
    __threadfence_block();
    __syncthreads();

    // ---------------------------------------------------------------- iterations
    StopController ctl(P.stop, P.tol);
    int cur = 0, best0 = -1, best1 = -1, best_j = -1;
    int rsj[2] = {-1, -1};
    double xn_prev = 0.0, xn_hist_a = 0.0, xn_hist_b = 0.0;  // ||X|| of the best pair
    double xn_last = 0.0, xn_last2 = 0.0;
    int done_buf = -1;
    for (int j = 1; j <= P.max_iter + 1; ++j) {
      if (j > P.max_iter) {
        info.reason = 2;
        info.status = -4;
        info.iters = P.max_iter;
        info.returned = P.max_iter;
        done_buf = cur;
        break;
      }
      int nxt = 0;
      while (nxt == cur || nxt == best0 || nxt == best1) ++nxt;
      const DM& Xc = X[cur];
      const DM& Xn = X[nxt];
      auto prod = [&](const DEpi& e) {
        double t0, t1;
        if (left)
          wg_gemm<MM, BM, BN, BK, WM, WN>(Xc, A, e, smem, sh, t0, t1);
        else
          wg_gemm<MM, BM, BN, BK, WM, WN>(A, Xc, e, smem, sh, t0, t1);
      };
      double sd = 0.0, sx = 0.0;
      auto apply = [&](const DM& T) {
        DEpi e = epi_out(Xn);
        e.nin = 1;
        e.in[0] = Xc;
        e.ref = 0;
        e.reduce = 1;
        if (left)
          wg_gemm<MM, BM, BN, BK, WM, WN>(T, Xc, e, smem, sh, sd, sx);
        else
          wg_gemm<MM, BM, BN, BK, WM, WN>(Xc, T, e, smem, sh, sd, sx);
      };
      const DM R = buf(0, s, s);
      double t0, t1;
      if (P.method == 0) {  // Newton-Schulz: T = 2I - prod (R = I - prod kept for the stop rule)
        const DM T = buf(1, s, s);
        DEpi e = epi_out(T, -1.f, 2.f);
        e.nout = 2;
        e.out[1] = R;
        e.a[1] = -1.f;
        e.g[1] = 1.f;
        prod(e);
        apply(T);
      } else if (P.method == 2) {  // QSAI
        const DM Sp = buf(1, s, s), R2 = buf(2, s, s), P1 = buf(3, s, s), P2 = buf(4, s, s), Qm = buf(5, s, s);
        DEpi e = epi_out(R, -1.f, 1.f);
        e.nout = 2;
        e.out[1] = Sp;
        e.a[1] = -1.f;
        e.g[1] = 2.f;
        prod(e);
        wg_gemm<MM, BM, BN, BK, WM, WN>(R, R, epi_out(R2), smem, sh, t0, t1);
        DEpi e4;
        e4.nout = 2;
        e4.out[0] = P1;
        e4.out[1] = P2;
        e4.nin = 1;
        e4.in[0] = R2;
        e4.b[0][0] = P.k.beta1;
        e4.b[1][0] = P.k.beta2;
        e4.g[0] = e4.g[1] = 1.f;
        wg_gemm<MM, BM, BN, BK, WM, WN>(R2, R2, e4, smem, sh, t0, t1);
        wg_gemm<MM, BM, BN, BK, WM, WN>(P1, P2, epi_out(Qm), smem, sh, t0, t1);
        wg_gemm<MM, BM, BN, BK, WM, WN>(Sp, Qm, epi_out(R2), smem, sh, t0, t1);
        apply(R2);
      } else {  // QHPI19 (Algorithm 3)
        const DM R2 = buf(1, s, s), R4 = buf(2, s, s), S = buf(3, s, s), P1 = buf(4, s, s), P2 = buf(5, s, s),
                 V = buf(6, s, s), Wm = buf(7, s, s);
        prod(epi_out(R, -1.f, 1.f));
        {
          DEpi e = epi_out(R2);
          e.nout = 2;
          e.out[1] = S;
          e.nin = 1;
          e.in[0] = R;
          e.b[1][0] = 1.f;
          wg_gemm<MM, BM, BN, BK, WM, WN>(R, R, e, smem, sh, t0, t1);
        }
        {
          DEpi e = epi_out(R4);
          e.nout = 3;
          e.out[1] = P1;
          e.out[2] = P2;
          e.nin = 1;
          e.in[0] = R2;
          e.b[1][0] = P.k.d1;
          e.b[2][0] = P.k.d2;
          e.g[1] = e.g[2] = 1.f;
          wg_gemm<MM, BM, BN, BK, WM, WN>(R2, R2, e, smem, sh, t0, t1);
        }
        {
          DEpi e;
          e.nout = 2;
          e.out[0] = V;
          e.out[1] = Wm;
          e.nin = 2;
          e.in[0] = R2;
          e.in[1] = R4;
          e.b[0][0] = P.k.d3;
          e.b[1][0] = P.k.e1;
          e.b[1][1] = P.k.e2;
          wg_gemm<MM, BM, BN, BK, WM, WN>(P1, P2, e, smem, sh, t0, t1);
        }
        {
          DEpi e = epi_out(P1);
          e.nin = 2;
          e.in[0] = R2;
          e.in[1] = R4;
          e.b[0][0] = P.k.c1;
          e.b[0][1] = P.k.c2;
          wg_gemm<MM, BM, BN, BK, WM, WN>(V, Wm, e, smem, sh, t0, t1);
        }
        wg_gemm<MM, BM, BN, BK, WM, WN>(S, P1, epi_out(P2, 1.f, 1.f), smem, sh, t0, t1);
        apply(P2);
      }
      // keep R_{j-1} (residual of X_{j-1}) for the candidate choice of the guarded rule
      const int rs = (j - 1) & 1;
      for (int e = tid; e < s * s; e += nthr) {
        const int i = e / s, c = e - i * s;
        for (int p = 0; p < 4; ++p) W[(int64_t)(BR + rs) * 4 * PS + p * PS + (int64_t)i * D + c] = R.p[p * PS + (int64_t)i * D + c];
      }
      __threadfence_block();
      __syncthreads();
      rsj[rs] = j - 1;

      const double d_abs = sqrt(fmax(sd, 0.0)), xn = sqrt(fmax(sx, 0.0));
      info.iters = j;
      info.dx_rel = xn > 0.0 ? d_abs / xn : 0.0;
      xn_last2 = xn_last;
      xn_last = xn;
      if (!__builtin_isfinite(d_abs) || !__builtin_isfinite(xn) || xn * normA > 1e20) {
        info.reason = 3;
        info.status = -3;
        info.returned = __builtin_isfinite(xn) ? j : j - 1;
        done_buf = __builtin_isfinite(xn) ? nxt : cur;
        break;
      }
      const int dec = ctl.update(j, d_abs, xn, -1.0);
      if (dec == D_TOL) {
        info.reason = 0;
        info.returned = j;
        done_buf = nxt;
        break;
      }
      if (dec == D_NEWMIN) {
        best0 = cur;
        best1 = nxt;
        best_j = j;
        xn_hist_a = xn_prev;
        xn_hist_b = xn;
      }
      if (dec == D_RISE) {
        info.reason = 1;
        const int ka = best_j - 1, kb = best_j;
        double ea = 1e300, eb = 1e300;
        if (rsj[ka & 1] == ka && rsj[kb & 1] == kb) {
          // X A X - X = -R X (left) or -X R (right)
          const DM Ra = buf(BR + (ka & 1), s, s), Rb = buf(BR + (kb & 1), s, s);
          const DM O = buf(BE, n, m);
          DEpi e = epi_out(O);
          e.reduce = 1;
          double q0, q1;
          if (left)
            wg_gemm<MM, BM, BN, BK, WM, WN>(Ra, X[best0], e, smem, sh, q0, q1);
          else
            wg_gemm<MM, BM, BN, BK, WM, WN>(X[best0], Ra, e, smem, sh, q0, q1);
          ea = sqrt(q0) / fmax(xn_hist_a, 1e-300);
          if (left)
            wg_gemm<MM, BM, BN, BK, WM, WN>(Rb, X[best1], e, smem, sh, q0, q1);
          else
            wg_gemm<MM, BM, BN, BK, WM, WN>(X[best1], Rb, e, smem, sh, q0, q1);
          eb = sqrt(q0) / fmax(xn_hist_b, 1e-300);
        }
        if (ka >= 1 && ea < eb) {
          info.returned = ka;
          done_buf = best0;
        } else {
          info.returned = kb;
          done_buf = best1;
        }
        break;
      }
      if (dec == D_DIVERGED) {
        info.reason = 3;
        info.status = -3;
        info.returned = j - 1;
        done_buf = cur;
        break;
      }
      xn_prev = xn;
      cur = nxt;
    }
    (void)xn_last2;
    // ---------------------------------------------------------------- result
    const DM& Xr = X[done_buf];
    for (int e = tid; e < n * m; e += nthr) {
      const int i = e / m, j = e - i * m;
      for (int p = 0; p < 4; ++p) d.X[p * d.psx + (int64_t)i * d.ldx + j] = Xr.p[p * PS + (int64_t)i * D + j];
    }
    if (tid == 0) P.info[b] = info;
    __threadfence();
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
using BatchedLaunch = void (*)(const BParams&, int grid, hipStream_t);

template <class MM, int BM, int BN, int BK, int WM, int WN>
static void launch_batched(const BParams& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL((batched_kernel<MM, BM, BN, BK, WM, WN>), dim3(grid), dim3(64 * WM * WN), 0, s, P);
  QP_HIP(hipGetLastError());
}

template <class MM, int BM, int BN, int BK, int WM, int WN>
static int occupancy_of() {
  int nb = 0;
  QP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_kernel<MM, BM, BN, BK, WM, WN>, 64 * WM * WN, 0));
  return std::max(nb, 1);
}

struct BatchedEntry {
  const char* name;
  BatchedLaunch fn;
  int (*occ)();
};

static const std::vector<BatchedEntry>& batched_table() {
  static const std::vector<BatchedEntry> t = {
      {"batched_f32_32x32x16_mfma16", launch_batched<MM16F, 32, 32, 16, 2, 2>, occupancy_of<MM16F, 32, 32, 16, 2, 2>},
      {"batched_f32_64x64x16_mfma32", launch_batched<MM32F, 64, 64, 16, 2, 2>, occupancy_of<MM32F, 64, 64, 16, 2, 2>},
      {"batched_f32_64x64x16_mfma16", launch_batched<MM16F, 64, 64, 16, 2, 2>, occupancy_of<MM16F, 64, 64, 16, 2, 2>},
  };
  return t;
}

int batched_num_configs() { return (int)batched_table().size(); }
const char* batched_config_name(int cfg) { return batched_table().at(cfg).name; }

__global__ void zero_int_kernel(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

BatchedState::~BatchedState() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (stream) (void)hipStreamDestroy(stream);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (h_desc) (void)hipHostFree(h_desc);
  if (h_info) (void)hipHostFree(h_info);
  if (h_order) (void)hipHostFree(h_order);
  if (h_alpha) (void)hipHostFree(h_alpha);
  for (void* p : dev) (void)hipFree(p);
}

static void* dev_alloc(BatchedState& st, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    throw Error(-6, "batched workspace allocation failed");
  }
  st.dev.push_back(p);
  return p;
}

// (Re)build device buffers and the captured graph for a batch signature.
static void build(BatchedState& st, const BKey& key, hipStream_t) {
  st.~BatchedState();
  new (&st) BatchedState();
  st.key = key;
  const int count = key.count, D = key.D;
  const auto& ent = batched_table().at(key.cfg);
  int dev = 0, cus = 0;
  QP_HIP(hipGetDevice(&dev));
  QP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // all workgroups resident; at most two per compute unit (bounds the per-workgroup scratch)
  st.grid = std::max(1, std::min({count, cus * ent.occ(), 2 * cus}));
  QP_HIP(hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking));
  QP_HIP(hipEventCreateWithFlags(&st.ev0, hipEventDisableTiming));
  QP_HIP(hipEventCreateWithFlags(&st.ev1, hipEventDisableTiming));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_desc), sizeof(BDesc) * count, hipHostMallocDefault));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_info), sizeof(BInfo) * count, hipHostMallocDefault));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_order), sizeof(int) * count, hipHostMallocDefault));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_alpha), sizeof(double) * count, hipHostMallocDefault));
  BDesc* d_desc = static_cast<BDesc*>(dev_alloc(st, sizeof(BDesc) * count));
  BInfo* d_info = static_cast<BInfo*>(dev_alloc(st, sizeof(BInfo) * count));
  int* d_order = static_cast<int*>(dev_alloc(st, sizeof(int) * count));
  int* d_queue = static_cast<int*>(dev_alloc(st, sizeof(int)));
  const int64_t PS = (int64_t)D * D;
  float* work = static_cast<float*>(dev_alloc(st, sizeof(float) * (size_t)st.grid * NBUF * 4 * PS));
  double* d_alpha = static_cast<double*>(dev_alloc(st, sizeof(double) * count));
  double* dwork = static_cast<double*>(dev_alloc(st, sizeof(double) * (size_t)st.grid * (8 * D + 64)));

  BParams P;
  P.desc = d_desc;
  P.info = d_info;
  P.order = d_order;
  P.count = count;
  P.queue = d_queue;
  P.work = work;
  P.dwork = dwork;
  P.D = D;
  P.method = key.method;
  P.stop = key.stop;
  P.max_iter = key.max_iter;
  P.tol = key.tol;
  P.scaling = key.scaling;
  P.power_steps = key.power_steps;
  P.seed = key.seed;
  P.k = make_coef();
  P.alpha = d_alpha;

  hipStream_t s = st.stream;
  QP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  QP_HIP(hipMemcpyAsync(d_desc, st.h_desc, sizeof(BDesc) * count, hipMemcpyHostToDevice, s));
  QP_HIP(hipMemcpyAsync(d_order, st.h_order, sizeof(int) * count, hipMemcpyHostToDevice, s));
  QP_HIP(hipMemcpyAsync(d_alpha, st.h_alpha, sizeof(double) * count, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, d_queue);
  ent.fn(P, st.grid, s);
  QP_HIP(hipMemcpyAsync(st.h_info, d_info, sizeof(BInfo) * count, hipMemcpyDeviceToHost, s));
  QP_HIP(hipStreamEndCapture(s, &st.graph));
  QP_HIP(hipGraphInstantiate(&st.exec, st.graph, nullptr, nullptr, 0));
}

void run_batched(BatchedState& st, const BKey& key, const std::vector<BDesc>& desc, const std::vector<int>& order,
                 const std::vector<double>& alphas, std::vector<BInfo>& infos, hipStream_t caller) {
  if (!st.exec || !(st.key == key)) build(st, key, caller);
  const int count = key.count;
  std::memcpy(st.h_desc, desc.data(), sizeof(BDesc) * count);
  std::memcpy(st.h_order, order.data(), sizeof(int) * count);
  for (int b = 0; b < count; ++b) st.h_alpha[b] = b < (int)alphas.size() ? alphas[b] : 0.0;
  // order the graph after the caller's stream, and the caller after the graph
  QP_HIP(hipEventRecord(st.ev0, caller));
  QP_HIP(hipStreamWaitEvent(st.stream, st.ev0, 0));
  QP_HIP(hipGraphLaunch(st.exec, st.stream));
  QP_HIP(hipEventRecord(st.ev1, st.stream));
  QP_HIP(hipStreamWaitEvent(caller, st.ev1, 0));
  QP_HIP(hipStreamSynchronize(st.stream));
  infos.assign(st.h_info, st.h_info + count);
}

}  // namespace qp

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

// Loads issued together per lane in the power iteration's row pass (fixed count, addresses clamped
// into A): a chunk of kSetupRows rows x 64 kSetupGroups columns then costs one memory latency.
constexpr int kSetupGroups = 2;
constexpr int kSetupRows = 4;

// sum over the 64 lanes of a wave, fixed order (every lane gets the total)
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Power iteration on A^H A with v (4 n doubles) and w (4 m doubles) in LDS, so that every load in
// flight is one of A's.  w = A v / ||v||: a wave takes kSetupRows rows at a time, lanes along them.
// v = A^H w: a wave takes 64 columns, lanes along them, and runs down all rows 8 at a time (no
// reduction across waves).  Returns ||w||^2 of the last step.
__device__ __forceinline__ double power_lds(const DM& A, int steps, unsigned long long seed, double* vs, double* ws,
                                            double* sh) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  const int m = A.rows, n = A.cols;
  constexpr int RR = kSetupRows, CG = kSetupGroups, RC = 8;
  for (int e = tid; e < 4 * n; e += nthr) vs[e] = (double)(bsplitmix64((uint64_t)e, seed) >> 11) * 0x1p-52 - 1.0;
  __syncthreads();
  double lam = 0.0;
  for (int step = 0; step < steps; ++step) {
    double nv = 0.0;
    for (int e = tid; e < 4 * n; e += nthr) nv += vs[e] * vs[e];
    nv = wg_sum(nv, sh);
    const double inv = 1.0 / sqrt(nv);
    for (int i0 = RR * wave; i0 < m; i0 += RR * nw) {
      double acc[RR][4];
#pragma unroll
      for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
      for (int j0 = 0; j0 < n; j0 += 64 * CG) {
        float a[RR][CG][4];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          const int64_t i = i0 + r < m ? i0 + r : m - 1;
#pragma unroll
          for (int k = 0; k < CG; ++k) {
            const int j = j0 + lane + 64 * k;
            const int64_t o = i * A.ld + (j < n ? j : n - 1);
#pragma unroll
            for (int p = 0; p < 4; ++p) a[r][k][p] = gload(A.p, p * A.ps + o);
          }
        }
#pragma unroll
        for (int k = 0; k < CG; ++k) {
          const int j = j0 + lane + 64 * k;
          const bool ok = j < n;
          const int jc = ok ? j : 0;
          const double vs0 = ok ? vs[jc] : 0.0, vx = ok ? vs[n + jc] : 0.0, vy = ok ? vs[2 * n + jc] : 0.0,
                       vz = ok ? vs[3 * n + jc] : 0.0;
#pragma unroll
          for (int r = 0; r < RR; ++r) {
            const double as = a[r][k][0], ax = a[r][k][1], ay = a[r][k][2], az = a[r][k][3];
            acc[r][0] += as * vs0 - ax * vx - ay * vy - az * vz;
            acc[r][1] += as * vx + ax * vs0 + ay * vz - az * vy;
            acc[r][2] += as * vy - ax * vz + ay * vs0 + az * vx;
            acc[r][3] += as * vz + ax * vy - ay * vx + az * vs0;
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double t = wave_sum(acc[r][c]);
          if (lane == 0 && i0 + r < m) ws[c * m + i0 + r] = t * inv;
        }
    }
    __syncthreads();
    double l2 = 0.0;
    for (int e = tid; e < 4 * m; e += nthr) l2 += ws[e] * ws[e];
    lam = wg_sum(l2, sh);
    for (int c0 = 64 * wave; c0 < n; c0 += 64 * nw) {
      const int j = c0 + lane;
      const int jc = j < n ? j : n - 1;
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
      for (int i0 = 0; i0 < m; i0 += RC) {
        float a[RC][4];
#pragma unroll
        for (int r = 0; r < RC; ++r) {
          const int64_t o = (int64_t)(i0 + r < m ? i0 + r : m - 1) * A.ld + jc;
#pragma unroll
          for (int p = 0; p < 4; ++p) a[r][p] = gload(A.p, p * A.ps + o);
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
          const int i = i0 + r;
          const bool ok = i < m;
          const int ic = ok ? i : 0;
          const double w0 = ok ? ws[ic] : 0.0, wx = ok ? ws[m + ic] : 0.0, wy = ok ? ws[2 * m + ic] : 0.0,
                       wz = ok ? ws[3 * m + ic] : 0.0;
          const double as = a[r][0], ax = a[r][1], ay = a[r][2], az = a[r][3];
          t0 += as * w0 + ax * wx + ay * wy + az * wz;
          t1 += as * wx - ax * w0 - ay * wz + az * wy;
          t2 += as * wy + ax * wz - ay * w0 - az * wx;
          t3 += as * wz - ax * wy + ay * wx - az * w0;
        }
      }
      if (j < n) {
        vs[j] = t0;
        vs[n + j] = t1;
        vs[2 * n + j] = t2;
        vs[3 * n + j] = t3;
      }
    }
    __syncthreads();
  }
  return lam;
}

// Power iteration on A^H A in ONE pass over A per step, for n <= 64 PF_CH: lanes along the columns (chunk k
// of a lane is column lane + 64 k), v in registers.  For a batch of PF_ROWS rows of a wave, w_i = (A v)_i /
// ||v|| is the wave sum of the lanes' partial products, and each lane then adds conj(a_ij) w_i into its
// columns of A^H w while the row is still in registers; the waves' partial A^H w are added in wave order
// through LDS.  Half the reads of the two-pass form.  (Loading the next batch during this one's arithmetic
// needs a second batch of registers, which the kernel's budget does not leave.)
// vs: 4 n doubles; red: (waves) 4 x 64 doubles.  Returns ||w||^2 of the last step.
constexpr int PF_CH = 4, PF_ROWS = 2;
__device__ __forceinline__ double power_fused(const DM& A, int steps, unsigned long long seed, double* vs, double* red,
                                              double* sh) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  const int m = A.rows, n = A.cols;
  for (int e = tid; e < 4 * n; e += nthr) vs[e] = (double)(bsplitmix64((uint64_t)e, seed) >> 11) * 0x1p-52 - 1.0;
  __syncthreads();
  double lam = 0.0;
  for (int step = 0; step < steps; ++step) {
    double nv = 0.0;
    for (int e = tid; e < 4 * n; e += nthr) nv += vs[e] * vs[e];
    nv = wg_sum(nv, sh);
    const double inv = 1.0 / sqrt(nv);
    double vr[PF_CH][4], acc[PF_CH][4];
#pragma unroll
    for (int k = 0; k < PF_CH; ++k) {
      const int j = lane + 64 * k;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        vr[k][p] = j < n ? vs[p * n + j] : 0.0;  // zero outside A: the clamped loads there add nothing to w
        acc[k][p] = 0.0;
      }
    }
    double l2 = 0.0;
    for (int i0 = PF_ROWS * wave; i0 < m; i0 += PF_ROWS * nw) {
      float a[PF_ROWS][PF_CH][4];
#pragma unroll
      for (int r = 0; r < PF_ROWS; ++r) {
        const int64_t i = i0 + r < m ? i0 + r : m - 1;
#pragma unroll
        for (int k = 0; k < PF_CH; ++k) {
          const int j = lane + 64 * k;
          const int64_t o = i * A.ld + (j < n ? j : n - 1);
#pragma unroll
          for (int p = 0; p < 4; ++p) a[r][k][p] = gload(A.p, p * A.ps + o);
        }
      }
#pragma unroll
      for (int r = 0; r < PF_ROWS; ++r) {
        double w[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < PF_CH; ++k) {
          const double as = a[r][k][0], ax = a[r][k][1], ay = a[r][k][2], az = a[r][k][3];
          const double v0 = vr[k][0], vx = vr[k][1], vy = vr[k][2], vz = vr[k][3];
          w[0] += as * v0 - ax * vx - ay * vy - az * vz;
          w[1] += as * vx + ax * v0 + ay * vz - az * vy;
          w[2] += as * vy - ax * vz + ay * v0 + az * vx;
          w[3] += as * vz + ax * vy - ay * vx + az * v0;
        }
        const bool rin = i0 + r < m;
#pragma unroll
        for (int c = 0; c < 4; ++c) w[c] = rin ? wave_sum(w[c]) * inv : 0.0;
        l2 += w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
#pragma unroll
        for (int k = 0; k < PF_CH; ++k) {
          const double as = a[r][k][0], ax = a[r][k][1], ay = a[r][k][2], az = a[r][k][3];
          acc[k][0] += as * w[0] + ax * w[1] + ay * w[2] + az * w[3];
          acc[k][1] += as * w[1] - ax * w[0] - ay * w[3] + az * w[2];
          acc[k][2] += as * w[2] + ax * w[3] - ay * w[0] - az * w[1];
          acc[k][3] += as * w[3] - ax * w[2] + ay * w[1] - az * w[0];
        }
      }
    }
    lam = wg_sum(lane == 0 ? l2 : 0.0, sh);  // every lane of a wave holds the wave's sum
#pragma unroll
    for (int k = 0; k < PF_CH; ++k) {
      if (64 * k >= n) break;
#pragma unroll
      for (int p = 0; p < 4; ++p) red[(wave * 4 + p) * 64 + lane] = acc[k][p];
      __syncthreads();
      for (int e = tid; e < 4 * 64; e += nthr) {
        const int p = e >> 6, l = e & 63, j = 64 * k + l;
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += red[(q * 4 + p) * 64 + l];
        if (j < n) vs[p * n + j] = t;
      }
      __syncthreads();
    }
  }
  return lam;
}

// Per-matrix set-up by one workgroup: finiteness and ||A||_F, the scaling (power iteration on A^H A
// from the SplitMix64 start vector, or the given alpha) and X_0 = alpha A^H into X0; A is also copied
// to Ac unless Ac.p is null.  The power iteration keeps its vectors in `lds` (lds_floats floats) when
// they fit, else in `dw` (4 (Dv + Dv) doubles with Dv >= max(m, n)).  Returns false (info.status =
// ENONFINITE) for a non-finite A.
__device__ __forceinline__ bool setup_matrix(int scaling, int power_steps, unsigned long long seed, double alpha_given,
                                             const DM& A, const DM& Ac, const DM& X0, double* dw, int Dv, double* sh,
                                             float* lds, int lds_floats, BInfo& info, double& normA, double& alpha) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int lane = tid & 63, nw = nthr >> 6;
  const int m = A.rows, n = A.cols;
  // one wave per row, lanes along the row: coalesced, 4 chunks of 64 columns in flight per wave
  constexpr int NG = 4;
  double fro2 = 0.0, nf = 0.0;
  for (int i = tid >> 6; i < m; i += nw) {
    for (int j0 = 0; j0 < n; j0 += 64 * NG) {
      float a[NG][4];
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        const int j = j0 + lane + 64 * k;
        const bool ok = j < n;
        const int64_t o = (int64_t)i * A.ld + (ok ? j : n - 1);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const float x = gload(A.p, p * A.ps + o);
          a[k][p] = ok ? x : 0.f;
        }
      }
      if (Ac.p != nullptr) {
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          const int j = j0 + lane + 64 * k;
          if (j < n)
#pragma unroll
            for (int p = 0; p < 4; ++p) gstore(Ac.p, p * Ac.ps + (int64_t)i * Ac.ld + j, a[k][p]);
        }
      }
#pragma unroll
      for (int k = 0; k < NG; ++k) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const double v = a[k][p];
          if (!__builtin_isfinite(v)) nf += 1.0;
          fro2 += v * v;
        }
      }
    }
  }
  fro2 = wg_sum(fro2, sh);
  nf = wg_sum(nf, sh);
  if (nf > 0.0) {
    info.status = -2;
    return false;
  }
  normA = sqrt(fro2);
  if (scaling == 2) {
    alpha = alpha_given;
  } else if (n <= 64 * PF_CH && 8 * n + 512 * nw <= lds_floats) {
    const double lam = power_fused(A, power_steps, seed, reinterpret_cast<double*>(lds),
                                   reinterpret_cast<double*>(lds) + 4 * n, sh);
    info.sigma1_sq = lam;
    alpha = 1.0 / lam;
  } else if (8 * (m + n) <= lds_floats) {
    const double lam = power_lds(A, power_steps, seed, reinterpret_cast<double*>(lds),
                                 reinterpret_cast<double*>(lds) + 4 * n, sh);
    info.sigma1_sq = lam;
    alpha = 1.0 / lam;
  } else {
    double* v = dw;            // 4n
    double* wv = dw + 4 * Dv;  // 4m
    for (int e = tid; e < 4 * n; e += nthr) v[e] = (double)(bsplitmix64((uint64_t)e, seed) >> 11) * 0x1p-52 - 1.0;
    __syncthreads();
    double lam = 0.0;
    for (int k = 0; k < power_steps; ++k) {
      double nv = 0.0;
      for (int e = tid; e < 4 * n; e += nthr) nv += v[e] * v[e];
      nv = wg_sum(nv, sh);
      const double inv = 1.0 / sqrt(nv);
      // w = A v: one wave per row, lanes along the row (coalesced), fixed-order wave reduction; NG
      // column chunks in flight per row.
      for (int i = tid >> 6; i < m; i += nw) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int j0 = 0; j0 < n; j0 += 64 * NG) {
          float a[NG][4];
          double vv[NG][4];
#pragma unroll
          for (int k = 0; k < NG; ++k) {
            const int j = j0 + lane + 64 * k;
            const bool ok = j < n;
            const int64_t o = (int64_t)i * A.ld + (ok ? j : 0);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              const float x = gload(A.p, p * A.ps + o);
              const double y = gload(v, p * n + (ok ? j : 0));
              a[k][p] = ok ? x : 0.f;
              vv[k][p] = ok ? y : 0.0;
            }
          }
#pragma unroll
          for (int k = 0; k < NG; ++k) {
            const double as = a[k][0], ax = a[k][1], ay = a[k][2], az = a[k][3];
            const double vs = vv[k][0], vx = vv[k][1], vy = vv[k][2], vz = vv[k][3];
            s0 += as * vs - ax * vx - ay * vy - az * vz;
            s1 += as * vx + ax * vs + ay * vz - az * vy;
            s2 += as * vy - ax * vz + ay * vs + az * vx;
            s3 += as * vz + ax * vy - ay * vx + az * vs;
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          s0 += __shfl_xor(s0, off, 64);
          s1 += __shfl_xor(s1, off, 64);
          s2 += __shfl_xor(s2, off, 64);
          s3 += __shfl_xor(s3, off, 64);
        }
        if (lane == 0) {
          wv[i] = s0 * inv;
          wv[m + i] = s1 * inv;
          wv[2 * m + i] = s2 * inv;
          wv[3 * m + i] = s3 * inv;
        }
      }
      __syncthreads();
      double l2 = 0.0;
      for (int e = tid; e < 4 * m; e += nthr) l2 += wv[e] * wv[e];
      lam = wg_sum(l2, sh);
      // v = A^H w: lanes along 64 columns (coalesced), the waves split the rows; the waves' partial
      // sums are added in wave order through LDS
      double* red = reinterpret_cast<double*>(lds);  // [waves][64][4]
      for (int j0 = 0; j0 < n; j0 += 64) {
        const int j = j0 + lane;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (j < n) {
          // rows i0 + k nw, k < NG, loaded together (fixed count, predicated)
          for (int i0 = tid >> 6; i0 < m; i0 += NG * nw) {
            float a[NG][4];
            double ww[NG][4];
#pragma unroll
            for (int k = 0; k < NG; ++k) {
              const int i = i0 + k * nw;
              const bool ok = i < m;
              const int64_t o = (int64_t)(ok ? i : 0) * A.ld + j;
#pragma unroll
              for (int p = 0; p < 4; ++p) {
                const float x = gload(A.p, p * A.ps + o);
                const double y = gload(wv, p * m + (ok ? i : 0));
                a[k][p] = ok ? x : 0.f;
                ww[k][p] = ok ? y : 0.0;
              }
            }
#pragma unroll
            for (int k = 0; k < NG; ++k) {
              const double as = a[k][0], ax = a[k][1], ay = a[k][2], az = a[k][3];
              const double ws = ww[k][0], wx = ww[k][1], wy = ww[k][2], wz = ww[k][3];
              s0 += as * ws + ax * wx + ay * wy + az * wz;
              s1 += as * wx - ax * ws - ay * wz + az * wy;
              s2 += as * wy + ax * wz - ay * ws - az * wx;
              s3 += as * wz - ax * wy + ay * wx - az * ws;
            }
          }
        }
        double* r = red + (int64_t)(tid >> 6) * 256 + lane * 4;
        r[0] = s0;
        r[1] = s1;
        r[2] = s2;
        r[3] = s3;
        __syncthreads();
        if (tid < 64 && j < n) {
          double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
          for (int q = 0; q < nw; ++q) {
            const double* rq = red + q * 256 + lane * 4;
            t0 += rq[0];
            t1 += rq[1];
            t2 += rq[2];
            t3 += rq[3];
          }
          v[j] = t0;
          v[n + j] = t1;
          v[2 * n + j] = t2;
          v[3 * n + j] = t3;
        }
        __syncthreads();
      }
    }
    info.sigma1_sq = lam;
    alpha = 1.0 / lam;
  }
  info.alpha = alpha;
  // X_0 = alpha A^H, transposed through 32 x 32 LDS tiles of all four planes (coalesced reads and writes).
  // A thread's rows of a tile (up to XR of them, all four planes) are loaded before any is stored, one
  // memory latency per tile; addresses are clamped into A and the values outside it replaced by zeros.
  constexpr int XR = 4;
  float* tile = lds;  // [4][32][33]
  const int tr = tid >> 5, tc = tid & 31, rstep = nthr >> 5;
  for (int ib = 0; ib < m; ib += 32)
    for (int jb = 0; jb < n; jb += 32) {
      for (int r0 = tr; r0 < 32; r0 += XR * rstep) {
        float x[XR][4];
#pragma unroll
        for (int u = 0; u < XR; ++u) {
          const int i = ib + r0 + u * rstep, j = jb + tc;
          const int64_t o = (int64_t)(i < m ? i : m - 1) * A.ld + (j < n ? j : n - 1);
#pragma unroll
          for (int p = 0; p < 4; ++p) x[u][p] = gload(A.p, p * A.ps + o);
        }
#pragma unroll
        for (int u = 0; u < XR; ++u) {
          const int r = r0 + u * rstep, i = ib + r, j = jb + tc;
          if (r < 32) {
            const bool ok = i < m && j < n;
#pragma unroll
            for (int p = 0; p < 4; ++p) tile[(p * 32 + r) * 33 + tc] = ok ? x[u][p] : 0.f;
          }
        }
      }
      __syncthreads();
      for (int r = tr; r < 32; r += rstep) {
        const int j = jb + r, i = ib + tc;
        if (j < n && i < m) {
#pragma unroll
          for (int p = 0; p < 4; ++p)
            gstore(X0.p, p * X0.ps + (int64_t)j * X0.ld + i,
                   (float)((p == 0 ? alpha : -alpha) * (double)tile[(p * 32 + tc) * 33 + r]));
        }
      }
      __syncthreads();
    }
  __threadfence_block();
  __syncthreads();
  return true;
}

template <class MM, int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) batched_kernel(BParams P) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) float smem[C::SMEM];
  static_assert(C::SMEM >= 4 * 32 * 33 && C::SMEM >= 2 * 4 * 64 * 4, "set-up scratch fits in the staging LDS");
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

    DM X[4] = {buf(BX, n, m), buf(BX + 1, n, m), buf(BX + 2, n, m), buf(BX + 3, n, m)};
    double normA = 0.0, alpha = 0.0;
    DM none;
    none.p = nullptr;
    if (!setup_matrix(P.scaling, P.power_steps, P.seed, P.scaling == 2 ? P.alpha[b] : 0.0, A, none, X[0], dw, D, sh, smem,
                      C::SMEM,
                      info, normA, alpha)) {
      if (tid == 0) P.info[b] = info;
      continue;
    }

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
        for (int p = 0; p < 4; ++p)
          gstore(W, (int64_t)(BR + rs) * 4 * PS + p * PS + (int64_t)i * D + c, gload(R.p, p * PS + (int64_t)i * D + c));
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
      for (int p = 0; p < 4; ++p) gstore(d.X, p * d.psx + (int64_t)i * d.ldx + j, gload(Xr.p, p * PS + (int64_t)i * D + j));
    }
    if (tid == 0) P.info[b] = info;
    __threadfence();
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------------
// Phase-synchronous form: all matrices advance one product of the method at a time.  Each phase's
// work items are the output tiles of that product over every still-active matrix; the workgroups
// (all resident: the grid is at most the occupancy times the compute units) take items i, i + G, ...,
// then meet at a grid barrier.  After the update phase a controller phase (one workgroup per active
// matrix) sums the update's per-tile change norms in tile order, applies the stop rule and either
// retires the matrix (copying its chosen iterate out) or moves it to the next update.  A large matrix
// is thus spread over many compute units instead of one, and small ones fill the gaps.
//
// The grid barrier is a counter and a generation word in device memory; arrival releases this
// workgroup's writes at device scope and leaving acquires the others'.  Every wait is bounded: a
// workgroup that waits too long raises the flag, and every workgroup leaves at the next barrier it
// sees the flag at, so the grid always drains.
// ------------------------------------------------------------------------------------------------
struct LState {
  int active, status, reason, returned;
  int pending;   // 1: the two candidate products of the rise rule are due (phases 1 and 2)
  int copy_buf;  // >= 0: copy this iterate to the caller's X in phase 1 of the next pass, then retire
  int j;  // updates done; the current iterate is X_j
  int cur, best0, best1, best_j;
  int rsj0, rsj1;  // iterates whose residuals the R buffers 0 and 1 hold
  unsigned int base;  // work items of this matrix completed before the current update (dataflow form)
  double alpha, normA, sigma1_sq, xn_prev, xn_a, xn_b, dx_rel;
  StopController ctl;
};

struct SParams {
  const BDesc* desc;
  BInfo* info;
  LState* st;
  int count;
  float* pool;
  double* partial;
  double* dwork;
  unsigned int* bar;  // [0] group arrivals, [1] generation, [2] timeout flag, [BAR_GROUP + 64 g] arrivals of group g
  const double* alpha;
  int method, stop, max_iter;
  double tol;
  int scaling, power_steps;
  unsigned long long seed;
  Coef k;
  unsigned long long* trace;  // optional: workgroup 0 stamps wall_clock64() after every grid barrier
  int trace_cap;
  unsigned int* qctr;  // per phase of the launch: the next work item (zeroed before the launch)
  int qctr_cap;        // phases with a counter; later phases (and dyn == 0) deal items g, g + G, ...
  int dyn;
  unsigned int* done;  // dataflow form: work items completed per matrix (zeroed before the launch)
};

constexpr int SYNC_MAX = 2048;   // matrices per launch (the per-phase tile prefix lives in LDS)
// Verbose trace of one launch (100 MHz wall-clock ticks): barrier stamps of workgroup 0 from 0, the per-matrix
// set-up durations from kTraceSetup, and every workgroup's time inside update work items from kTraceBusy.
constexpr int kTraceCap = 8192;
constexpr int kTraceSetup = 2048;
constexpr int kTraceBusy = 4096;
constexpr long long SPIN_MAX = 1ll << 22;  // barrier polls before the wait is abandoned

// Grid barrier; returns false once any workgroup has abandoned a wait.  Two levels: a workgroup arrives on
// its group's counter (group = blockIdx mod BAR_NG, the XCD it was dealt to; counters on separate 256-byte
// lines), the group's last arrival arrives on the global counter.  One counter taking every arrival
// serialises them at the memory side (measured 57 us per barrier for 512 workgroups, 25 us with the
// groups; 32 groups, or sleeping between polls, measured no faster).  The counters only grow during a solve
// (cleared before it): barrier k (the k-th of the solve, counted by every workgroup in `k`) is complete
// when group g's counter reaches k gsize and the global one k ngroups, so the last arrivals have nothing
// more to do than arrive.  Arrivals release this workgroup's writes; a group's last arrival acquires its
// group's (their adds form a release sequence) before it releases them on the global counter; every
// workgroup acquires once the global count is reached (its own add or a relaxed poll).  The give-up flag
// is read by every poll: a workgroup whose wait needs no poll learns of a give-up at its next wait.
constexpr int BAR_NG = 8, BAR_GROUP = 64, BAR_WORDS = BAR_GROUP + 64 * BAR_NG;
__device__ bool grid_sync(unsigned int* bar, unsigned int nblocks, unsigned int& k) {
  __shared__ int s_ok;
  __syncthreads();
  ++k;
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned int g = blockIdx.x % BAR_NG;
    const unsigned int gsize = nblocks / BAR_NG + ((nblocks % BAR_NG) > g ? 1u : 0u);
    const unsigned int ngroups = nblocks < (unsigned int)BAR_NG ? nblocks : (unsigned int)BAR_NG;
    const unsigned int target = k * ngroups;
    bool last = false;
    unsigned int* gw = &bar[BAR_GROUP + 64 * g];
    if (__hip_atomic_fetch_add(gw, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1u == k * gsize) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      last = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1u == target;
    }
    if (!last) {
      long long spins = 0;
      while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > SPIN_MAX) {
          __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Views of matrix b's work buffers: 10 of s x s (chain 0..7, residuals 8..9) and 5 of n x m (iterates
// 0..3, candidate product 4); when A's rows are not 16-byte aligned, a copy of A whose rows are
// (BDesc::ldap > 0) follows them.  All have 16-byte aligned rows and planes, so every product takes
// 16-byte operand loads.
struct MBufs {
  float* base;
  int64_t lds, pss, ldw, psw;
  int s, m, n;
  __device__ DM sq(int k) const {
    DM v;
    v.p = base + (int64_t)k * 4 * pss;
    v.ld = lds;
    v.ps = pss;
    v.rows = v.cols = s;
    return v;
  }
  __device__ DM xw(int k) const {
    DM v;
    v.p = base + 10 * 4 * pss + (int64_t)k * 4 * psw;
    v.ld = ldw;
    v.ps = psw;
    v.rows = n;
    v.cols = m;
    return v;
  }
};

__device__ __forceinline__ MBufs mbufs(const SParams& P, const BDesc& d) {
  MBufs B;
  B.base = P.pool + d.off;
  B.lds = d.lds;
  B.pss = d.pss;
  B.ldw = d.ldw;
  B.psw = d.psw;
  B.m = d.m;
  B.n = d.n;
  B.s = d.m > d.n ? d.n : d.m;
  return B;
}

__device__ __forceinline__ int num_phases(int method) { return method == 0 ? 2 : method == 2 ? 6 : 7; }

// The product of phase `ph` (1-based; the last one is the update) of matrix b with iterate X_cur into
// X_nxt: operands, output shape and epilogue.
__device__ __forceinline__ void phase_product(const SParams& P, const MBufs& B, const LState& S, int nxt, int ph, DM& Aop, DM& Bop,
                              DEpi& e) {
  const bool left = B.m > B.n;
  const DM Xc = B.xw(S.cur), Xn = B.xw(nxt);
  const DM R = B.sq(8 + (S.j & 1));
  const int np = num_phases(P.method);
  e = DEpi();
  if (ph == np) {  // update: T X (left) or X T (right), change norms against X_cur
    const DM T = P.method == 0 ? B.sq(1) : P.method == 2 ? B.sq(2) : B.sq(5);
    e = epi_out(Xn);
    e.nin = 1;
    e.in[0] = Xc;
    e.ref = 0;
    e.reduce = 1;
    Aop = left ? T : Xc;
    Bop = left ? Xc : T;
    return;
  }
  if (ph == 1) {  // side product: X A (left) or A X (right); the caller fills the A view
    Aop = Xc;  // placeholder, replaced by the caller
    Bop = Xc;
    if (P.method == 0) {  // T = 2I - prod, R = I - prod
      e = epi_out(B.sq(1), -1.f, 2.f);
      e.nout = 2;
      e.out[1] = R;
      e.a[1] = -1.f;
      e.g[1] = 1.f;
    } else if (P.method == 2) {  // R and Sp = 2I - prod
      e = epi_out(R, -1.f, 1.f);
      e.nout = 2;
      e.out[1] = B.sq(1);
      e.a[1] = -1.f;
      e.g[1] = 2.f;
    } else {
      e = epi_out(R, -1.f, 1.f);
    }
    return;
  }
  if (P.method == 2) {  // QSAI: R2 = R R; P1, P2 from R2 R2; Q = P1 P2; T = Sp Q
    if (ph == 2) {
      Aop = R;
      Bop = R;
      e = epi_out(B.sq(2));
    } else if (ph == 3) {
      Aop = B.sq(2);
      Bop = B.sq(2);
      e.nout = 2;
      e.out[0] = B.sq(3);
      e.out[1] = B.sq(4);
      e.nin = 1;
      e.in[0] = B.sq(2);
      e.b[0][0] = P.k.beta1;
      e.b[1][0] = P.k.beta2;
      e.g[0] = e.g[1] = 1.f;
    } else if (ph == 4) {
      Aop = B.sq(3);
      Bop = B.sq(4);
      e = epi_out(B.sq(5));
    } else {  // ph == 5
      Aop = B.sq(1);
      Bop = B.sq(5);
      e = epi_out(B.sq(2));
    }
    return;
  }
  // QHPI19 (Algorithm 3): R2 (+ S = R + R2); R4 (+ P1, P2); V, W from P1 P2; G = V W + ...; T = I + S G
  const DM R2 = B.sq(0), R4 = B.sq(2), Sm = B.sq(3), P1 = B.sq(4), P2 = B.sq(5), V = B.sq(6), W = B.sq(7);
  if (ph == 2) {
    Aop = R;
    Bop = R;
    e = epi_out(R2);
    e.nout = 2;
    e.out[1] = Sm;
    e.nin = 1;
    e.in[0] = R;
    e.b[1][0] = 1.f;
  } else if (ph == 3) {
    Aop = R2;
    Bop = R2;
    e = epi_out(R4);
    e.nout = 3;
    e.out[1] = P1;
    e.out[2] = P2;
    e.nin = 1;
    e.in[0] = R2;
    e.b[1][0] = P.k.d1;
    e.b[2][0] = P.k.d2;
    e.g[1] = e.g[2] = 1.f;
  } else if (ph == 4) {
    Aop = P1;
    Bop = P2;
    e.nout = 2;
    e.out[0] = V;
    e.out[1] = W;
    e.nin = 2;
    e.in[0] = R2;
    e.in[1] = R4;
    e.b[0][0] = P.k.d3;
    e.b[1][0] = P.k.e1;
    e.b[1][1] = P.k.e2;
  } else if (ph == 5) {
    Aop = V;
    Bop = W;
    e = epi_out(P1);
    e.nin = 2;
    e.in[0] = R2;
    e.in[1] = R4;
    e.b[0][0] = P.k.c1;
    e.b[0][1] = P.k.c2;
  } else {  // ph == 6
    Aop = Sm;
    Bop = P1;
    e = epi_out(P2, 1.f, 1.f);
  }
}

// Workgroup-uniform values built from loaded data move to scalar registers (every lane holds the
// same value), which keeps the per-item product parameters out of the vector register budget.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
template <class T>
__device__ __forceinline__ T* uni(T* p) {
  return reinterpret_cast<T*>(uni((int64_t)reinterpret_cast<uintptr_t>(p)));
}

__device__ __forceinline__ void make_uniform(GemmParams<float>& G) {
  G.A = uni(G.A);
  G.lda = uni(G.lda);
  G.psa = uni(G.psa);
  G.B = uni(G.B);
  G.ldb = uni(G.ldb);
  G.psb = uni(G.psb);
  G.M = uni(G.M);
  G.N = uni(G.N);
  G.K = uni(G.K);
  G.tiles_m = uni(G.tiles_m);
  G.tiles_n = uni(G.tiles_n);
  G.vec = uni(G.vec);
  G.nout = uni(G.nout);
  G.nin = uni(G.nin);
  G.ref = uni(G.ref);
  G.reduce = uni(G.reduce);
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    G.out[t] = uni(G.out[t]);
    G.ldo[t] = uni(G.ldo[t]);
    G.pso[t] = uni(G.pso[t]);
    G.in[t] = uni(G.in[t]);
    G.ldi[t] = uni(G.ldi[t]);
    G.psi[t] = uni(G.psi[t]);
    G.ca[t] = uni(G.ca[t]);
    G.cg[t] = uni(G.cg[t]);
#pragma unroll
    for (int u = 0; u < 3; ++u) G.cb[t][u] = uni(G.cb[t][u]);
  }
}

// GemmParams of C = Aop Bop with epilogue e (FP32 storage).
__device__ __forceinline__ GemmParams<float> gemm_params(const DM& Aop, const DM& Bop, const DEpi& e, int BM, int BN) {
  GemmParams<float> G;
  G.A = Aop.p;
  G.lda = Aop.ld;
  G.psa = Aop.ps;
  G.B = Bop.p;
  G.ldb = Bop.ld;
  G.psb = Bop.ps;
  G.M = Aop.rows;
  G.N = Bop.cols;
  G.K = Aop.cols;
  G.tiles_m = (G.M + BM - 1) / BM;
  G.tiles_n = (G.N + BN - 1) / BN;
  G.vec = ((Aop.ld | Aop.ps | Bop.ld | Bop.ps) & 3) == 0 && ((reinterpret_cast<uintptr_t>(Aop.p) | reinterpret_cast<uintptr_t>(Bop.p)) & 15) == 0;
  G.nout = e.nout;
  G.nin = e.nin;
  G.ref = e.ref;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    G.out[t] = e.out[t].p;
    G.ldo[t] = e.out[t].ld;
    G.pso[t] = e.out[t].ps;
    G.in[t] = e.in[t].p;
    G.ldi[t] = e.in[t].ld;
    G.psi[t] = e.in[t].ps;
    G.ca[t] = e.a[t];
    G.cg[t] = e.g[t];
#pragma unroll
    for (int u = 0; u < 3; ++u) G.cb[t][u] = e.b[t][u];
  }
  G.partial = nullptr;
  G.reduce = e.reduce;
  return G;
}

// Tile t of a product: 16-byte operand loads, edge tiles included, when both operands allow them (the
// work buffers always do; the caller's A only with a 16-byte multiple row stride), else element loads.
template <class MM, int BM, int BN, int BK, int WM, int WN>
__device__ __forceinline__ void tile_any(const GemmParams<float>& G, int t, float* smem, double& a0, double& a1) {
  if (G.vec)
    gemm_tile<MM, BM, BN, BK, WM, WN, 128, kLoadVec, false, true>(G, t / G.tiles_n, t % G.tiles_n, smem, a0, a1);
  else
    gemm_tile<MM, BM, BN, BK, WM, WN, 128, kLoadScalar, false, true>(G, t / G.tiles_n, t % G.tiles_n, smem, a0, a1);
}

template <int BM, int BN>
__device__ __forceinline__ int tiles_of(int rows, int cols) {
  return ((rows + BM - 1) / BM) * ((cols + BN - 1) / BN);
}

// next free iterate buffer: not the current one and not the pair kept around the smallest change
__device__ __forceinline__ int next_buf(const LState& S) {
  int nxt = 0;
  while (nxt == S.cur || nxt == S.best0 || nxt == S.best1) ++nxt;
  return nxt;
}

// Work items of matrix b in phase ph of an update (1-based; np + 1 is the controller), from the state the
// update started in (flags: 1 active, 2 rise-rule candidates due, 4 result copy due) and the tile counts of
// its s x s and n x m products.
__device__ __forceinline__ int phase_items(int flags, int ph, int np, int sq, int out) {
  if (!(flags & 1)) return 0;
  if (ph > np) return 1;
  if (flags & 4) return ph == 1 ? out : 0;
  if (flags & 2) return ph <= 2 ? out : 0;
  return ph == np ? out : sq;
}

// PER_CU: resident workgroups per compute unit the register allocation leaves room for (and the
// launch uses, at most).
// FLOW: the dataflow form, for the updates whose first phase has at most FLOW_ITEMS items per workgroup
// (the last few matrices; with many, the barrier form measured faster).  In such an update the workgroups
// meet at a grid barrier once (after the controllers) instead of after every phase: they take the phases'
// items in phase order, each phase
// from its own counter, and an item of phase ph of matrix b first waits until b's items of the earlier
// phases of the update are complete (a per-matrix counter of completed items, raised with release
// semantics after each item and polled, then acquired, before the item).  A workgroup only takes a phase's
// items once that phase's counter has run out, so every item an item waits for was taken earlier by a
// resident workgroup that waits only for still earlier items: the waits always end.  Each wait is bounded
// like the barrier's and raises the same give-up flag.
constexpr int FLOW_ITEMS = 6;
template <class MM, int BM, int BN, int BK, int WM, int WN, int PER_CU = 2, bool FLOW = false>
__global__ void __launch_bounds__(64 * WM * WN, PER_CU) batched_sync_kernel(SParams P) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) float smem[C::SMEM];
  static_assert(C::SMEM >= 4 * 32 * 33 && C::SMEM >= 2 * 4 * 64 * 4, "set-up scratch fits in the staging LDS");
  __shared__ double sh[16];
  __shared__ int pref[SYNC_MAX + 1];
  __shared__ int s_mn[SYNC_MAX];  // m | n << 16 per matrix
  __shared__ unsigned char s_fl[SYNC_MAX];  // state of each matrix at the start of the update (phase_items)
  __shared__ int s_total;
  __shared__ int s_item;
  __shared__ int s_dep;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const unsigned int G = gridDim.x;
  unsigned int nbar = 0;  // grid barriers passed in this solve
  const int np = num_phases(P.method);
  unsigned long long* const trace = (blockIdx.x == 0 && tid == 0) ? P.trace : nullptr;
  const int trace_cap = P.trace_cap < kTraceSetup ? P.trace_cap : kTraceSetup;
  int nstamp = 0;
  unsigned long long busy = 0;  // this workgroup's ticks inside update work items (verbose trace only)
#define QP_STAMP()                                            \
  do {                                                        \
    if (trace && nstamp < trace_cap) trace[nstamp] = wall_clock64(); \
    ++nstamp;                                                 \
  } while (0)
  QP_STAMP();

  for (int b = tid; b < P.count; b += nthr) s_mn[b] = P.desc[b].m | (P.desc[b].n << 16);

  // ---------------------------------------------------------------- set-up: one workgroup per matrix
  for (int b = blockIdx.x; b < P.count; b += G) {
    const BDesc d = P.desc[b];
    const MBufs B = mbufs(P, d);
    DM A;
    A.p = const_cast<float*>(d.A);
    A.ld = d.lda;
    A.ps = d.psa;
    A.rows = d.m;
    A.cols = d.n;
    BInfo info;
    info.iters = 0;
    info.returned = 0;
    info.reason = 0;
    info.status = 0;
    info.alpha = 0.0;
    info.dx_rel = 0.0;
    info.sigma1_sq = 0.0;
    double normA = 0.0, alpha = 0.0;
    const int Dv = d.m > d.n ? d.m : d.n;
    const unsigned long long t_set = wall_clock64();
    DM Ac = A;  // the copy of A with 16-byte aligned rows, when there is one
    Ac.p = d.ldap > 0 ? B.base + 10 * 4 * d.pss + 5 * 4 * d.psw : nullptr;
    Ac.ld = d.ldap;
    Ac.ps = d.psap;
    const bool ok = setup_matrix(P.scaling, P.power_steps, P.seed, P.scaling == 2 ? P.alpha[b] : 0.0, A, Ac, B.xw(0),
                                 P.dwork + d.doff, Dv, sh, smem, C::SMEM, info, normA, alpha);
    if (P.trace && tid == 0 && kTraceSetup + b < kTraceBusy) P.trace[kTraceSetup + b] = wall_clock64() - t_set;
    if (tid == 0) {
      LState S;
      S.active = ok ? 1 : 0;
      S.pending = 0;
      S.copy_buf = -1;
      S.status = info.status;
      S.reason = 0;
      S.returned = 0;
      S.j = 0;
      S.cur = 0;
      S.best0 = S.best1 = S.best_j = -1;
      S.rsj0 = S.rsj1 = -1;
      S.alpha = alpha;
      S.normA = normA;
      S.sigma1_sq = info.sigma1_sq;
      S.xn_prev = S.xn_a = S.xn_b = 0.0;
      S.base = 0u;
      S.dx_rel = 0.0;
      S.ctl = StopController(P.stop, P.tol);
      P.st[b] = S;
      if (!ok) P.info[b] = info;
    }
    __syncthreads();
  }
  if (!grid_sync(P.bar, G, nbar)) return;
  QP_STAMP();

  // ---------------------------------------------------------------- updates
  // max_iter updates, plus one pass for the rise rule's candidate products
  for (int it = 0; it <= P.max_iter + 1; ++it) {
    // the matrices' states as the update starts (the controllers change them only in its last phase)
    for (int b = tid; b < P.count; b += nthr) {
      const LState& Sb = P.st[b];
      s_fl[b] = (unsigned char)(Sb.active ? 1 | (Sb.pending ? 2 : 0) | (Sb.copy_buf >= 0 ? 4 : 0) : 0);
    }
    __syncthreads();
    int known_b = -1;         // thread 0 (dataflow form): matrix and phase whose earlier items this
    int known_ph = 0;         // workgroup has already seen complete (and acquired)
    bool flowu = false;       // this update runs in the dataflow form (the same choice in every workgroup)
    for (int ph = 1; ph <= np + 1; ++ph) {
      // tile counts of this phase over the active matrices (phase np + 1: one item per active matrix)
      const int per = (P.count + nthr - 1) / nthr;
      int loc = 0;
      for (int q = 0; q < per; ++q) {
        const int b = tid * per + q;
        int c = 0;
        if (b < P.count) {
          const int mb = s_mn[b] & 0xffff, nb = s_mn[b] >> 16;
          const int sd = mb > nb ? nb : mb;
          c = phase_items(s_fl[b], ph, np, tiles_of<BM, BN>(sd, sd), tiles_of<BM, BN>(nb, mb));
          pref[b + 1] = c;
        }
        loc += c;
      }
      // exclusive scan of the per-thread totals: inclusive scan within each wave (shuffles), the waves'
      // totals through LDS, then each thread's run (integer sums: the same result in any order)
      __syncthreads();
      if (tid == 0) pref[0] = 0;
      {
        __shared__ int wtot[16];
        const int lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
        int incl = loc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int y = __shfl_up(incl, off, 64);
          if (lane >= off) incl += y;
        }
        if (lane == 63) wtot[wv] = incl;
        __syncthreads();
        int base = 0, tot = 0;
        for (int q = 0; q < nwv; ++q) {
          const int t = wtot[q];
          base += q < wv ? t : 0;
          tot += t;
        }
        if (tid == 0) s_total = tot;
        int run = base + incl - loc;
        for (int q = 0; q < per; ++q) {
          const int b = tid * per + q;
          if (b < P.count) {
            const int c = pref[b + 1];
            pref[b + 1] = run + c;
            run += c;
          }
        }
      }
      __syncthreads();
      const int total = s_total;
      if (ph == 1 && total == 0) return;  // nothing active: every workgroup sees the same states
      if (ph == 1) flowu = FLOW && total <= FLOW_ITEMS * (int)G;
      // Work items of this phase.  Dynamic: a workgroup takes the next unclaimed item from the phase's
      // counter (asking for the following one as it starts an item, so the atomic's latency hides
      // behind the tile), which balances items of different K; static: items g, g + G, ...  Either way
      // every item is computed once, by code that does not depend on which workgroup runs it.
      const int seq = it * (np + 1) + (ph - 1);
      const bool dyn = P.dyn != 0 && seq < P.qctr_cap;
      unsigned int pre = 0u;  // thread 0: the item claimed for after the current one
      auto first_item = [&]() -> int {
        if (!dyn) return (int)blockIdx.x;
        if (tid == 0) s_item = (int)__hip_atomic_fetch_add(&P.qctr[seq], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        return s_item;
      };
      auto next_item = [&](int item) -> int {
        if (!dyn) return item + (int)G;
        __syncthreads();  // every thread has read s_item
        if (tid == 0) s_item = (int)pre;
        __syncthreads();
        return s_item;
      };
      unsigned long long t_item = 0;
      for (int item = first_item(); item < total; item = next_item(item)) {
        if (P.trace && tid == 0) {
          const unsigned long long now = wall_clock64();
          if (t_item) busy += now - t_item;
          t_item = now;
        }
        if (dyn && tid == 0) pre = __hip_atomic_fetch_add(&P.qctr[seq], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // matrix of this item: last b with pref[b] <= item
        int lo = 0, hi = P.count;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (pref[mid] <= item) lo = mid; else hi = mid;
        }
        const int b = lo;
        const int t = item - pref[b];
        const BDesc d = P.desc[b];
        const MBufs B = mbufs(P, d);
        LState S = P.st[b];
        if constexpr (FLOW) {
          if (flowu && ph >= 2) {
            // wait for matrix b's items of phases 1 .. ph - 1 of this update
            if (tid == 0) {
              int ok = 1;
              if (known_b != b || known_ph != ph) {
                const int sd = d.m > d.n ? d.n : d.m;
                const int sq = tiles_of<BM, BN>(sd, sd), out = tiles_of<BM, BN>(d.n, d.m);
                unsigned int need = S.base;
                for (int q = 1; q < ph; ++q) need += (unsigned int)phase_items(s_fl[b], q, np, sq, out);
                long long spins = 0;
                while (__hip_atomic_load(&P.done[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                  if (__hip_atomic_load(&P.bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                      ++spins > SPIN_MAX) {
                    __hip_atomic_store(&P.bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                  }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                known_b = b;
                known_ph = ph;
              }
              s_dep = ok;
            }
            __syncthreads();
            if (!s_dep) return;
          }
        }
        // matrix b's item is complete: count it (dataflow form)
        auto item_done = [&]() {
          if (flowu) {
            __syncthreads();
            if (tid == 0) __hip_atomic_fetch_add(&P.done[b], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          }
        };
        if (ph <= np && S.copy_buf >= 0) {
          // tile t of the chosen iterate to the caller's X
          const DM Xr = B.xw(S.copy_buf);
          const int tn = (d.m + BN - 1) / BN;
          const int r0 = (t / tn) * BM, c0 = (t % tn) * BN;
          for (int e = tid; e < BM * BN; e += nthr) {
            const int i = r0 + e / BN, c = c0 + e % BN;
            if (i < d.n && c < d.m)
#pragma unroll
              for (int p = 0; p < 4; ++p)
                gstore(d.X, p * d.psx + (int64_t)i * d.ldx + c, gload(Xr.p, p * Xr.ps + (int64_t)i * Xr.ld + c));
          }
          item_done();
          continue;
        }
        if (ph <= np && S.pending) {
          // candidate product ph of the rise rule: R_k X_k (left) or X_k R_k (right), k = best_j - 1, best_j
          const bool left = d.m > d.n;
          const int kc = ph == 1 ? S.best_j - 1 : S.best_j;
          const DM Rr = B.sq(8 + (kc & 1));
          const DM Xr = B.xw(ph == 1 ? S.best0 : S.best1);
          DEpi eo = epi_out(B.xw(4));
          eo.reduce = 1;
          GemmParams<float> Gp = left ? gemm_params(Rr, Xr, eo, BM, BN) : gemm_params(Xr, Rr, eo, BM, BN);
          make_uniform(Gp);
          double a0 = 0.0, a1 = 0.0;
          tile_any<MM, BM, BN, BK, WM, WN>(Gp, t, smem, a0, a1);
          a0 = wg_sum(a0, sh);
          if (tid == 0) P.partial[d.poff + 2 * ((ph - 1) * tiles_of<BM, BN>(d.n, d.m) + t)] = a0;
          __syncthreads();
          item_done();
          continue;
        }
        if (ph <= np) {
          DM Aop, Bop;
          DEpi e;
          const int nxt = next_buf(S);
          phase_product(P, B, S, nxt, ph, Aop, Bop, e);
          if (ph == np) {  // the new iterate also goes to the caller's X (the result unless the rise rule picks)
            e.nout = 2;
            e.out[1].p = d.X;
            e.out[1].ld = d.ldx;
            e.out[1].ps = d.psx;
            e.a[1] = 1.f;
          }
          if (ph == 1) {
            const bool copied = d.ldap > 0;
            DM A;
            A.p = copied ? B.base + 10 * 4 * d.pss + 5 * 4 * d.psw : const_cast<float*>(d.A);
            A.ld = copied ? d.ldap : d.lda;
            A.ps = copied ? d.psap : d.psa;
            A.rows = d.m;
            A.cols = d.n;
            const DM Xc = B.xw(S.cur);
            const bool left = d.m > d.n;
            Aop = left ? Xc : A;
            Bop = left ? A : Xc;
          }
          GemmParams<float> Gp = gemm_params(Aop, Bop, e, BM, BN);
          make_uniform(Gp);
          double a0 = 0.0, a1 = 0.0;
          tile_any<MM, BM, BN, BK, WM, WN>(Gp, t, smem, a0, a1);
          if (ph == np) {
            a0 = wg_sum(a0, sh);
            a1 = wg_sum(a1, sh);
            if (tid == 0) {
              P.partial[d.poff + 2 * t] = a0;
              P.partial[d.poff + 2 * t + 1] = a1;
            }
          }
          __syncthreads();
          item_done();
          continue;
        }
        // ---------------------------------------------------------------- controller of matrix b
        const int nxt = next_buf(S);
        const int ntile = tiles_of<BM, BN>(d.n, d.m);
        if (flowu) {  // this update's items of matrix b, counted for the next dataflow update's waits
          const int sd = d.m > d.n ? d.n : d.m;
          for (int q = 1; q <= np; ++q)
            S.base += (unsigned int)phase_items(s_fl[b], q, np, tiles_of<BM, BN>(sd, sd), ntile);
        }
        if (S.copy_buf >= 0) {  // the copy ran in phase 1 of this pass
          S.copy_buf = -1;
          S.active = 0;
          if (tid == 0) {
            BInfo info;
            info.iters = S.j;
            info.returned = S.returned;
            info.reason = S.reason;
            info.status = S.status;
            info.alpha = S.alpha;
            info.dx_rel = S.dx_rel;
            info.sigma1_sq = S.sigma1_sq;
            P.info[b] = info;
            P.st[b] = S;
          }
          __syncthreads();
          continue;
        }
        if (S.pending) {
          // finish the rise rule: the better of X_{best_j - 1}, X_{best_j} by ||XAX - X||_F / ||X||_F
          double qa = 0.0, qb = 0.0;
          for (int q = tid; q < ntile; q += nthr) {
            qa += P.partial[d.poff + 2 * q];
            qb += P.partial[d.poff + 2 * (ntile + q)];
          }
          qa = wg_sum(qa, sh);
          qb = wg_sum(qb, sh);
          const double ea = sqrt(qa) / fmax(S.xn_a, 1e-300), eb = sqrt(qb) / fmax(S.xn_b, 1e-300);
          const int ka = S.best_j - 1;
          const int done_buf = (ka >= 1 && ea < eb) ? S.best0 : S.best1;
          S.returned = (ka >= 1 && ea < eb) ? ka : S.best_j;
          S.pending = 0;
          S.copy_buf = done_buf;  // an older iterate: copied in the next pass
          if (tid == 0) P.st[b] = S;
          __syncthreads();
          continue;
        }
        double sd0 = 0.0, sx0 = 0.0;
        for (int q = tid; q < ntile; q += nthr) {
          sd0 += P.partial[d.poff + 2 * q];
          sx0 += P.partial[d.poff + 2 * q + 1];
        }
        const double sdv = wg_sum(sd0, sh), sxv = wg_sum(sx0, sh);
        const double d_abs = sqrt(fmax(sdv, 0.0)), xn = sqrt(fmax(sxv, 0.0));
        const int j = S.j + 1;  // index of the new iterate X_j = buffer nxt
        if (S.j & 1)  // this update's residual belongs to X_{j-1}
          S.rsj1 = S.j;
        else
          S.rsj0 = S.j;
        S.dx_rel = xn > 0.0 ? d_abs / xn : 0.0;
        int done_buf = -1;
        if (!__builtin_isfinite(d_abs) || !__builtin_isfinite(xn) || xn * S.normA > 1e20) {
          S.reason = 3;
          S.status = -3;
          S.returned = __builtin_isfinite(xn) ? j : j - 1;
          done_buf = __builtin_isfinite(xn) ? nxt : S.cur;
        } else {
          const int dec = S.ctl.update(j, d_abs, xn, -1.0);
          if (dec == D_TOL) {
            S.reason = 0;
            S.returned = j;
            done_buf = nxt;
          } else if (dec == D_RISE) {
            S.reason = 1;
            const int ka = S.best_j - 1, kb = S.best_j;
            const int ra = (ka & 1) ? S.rsj1 : S.rsj0, rb = (kb & 1) ? S.rsj1 : S.rsj0;
            if (ka >= 0 && ra == ka && rb == kb) {
              S.pending = 1;  // the candidate products run in the next pass over the phases
            } else {
              S.returned = kb;
              done_buf = S.best1;
            }
          } else if (dec == D_DIVERGED) {
            S.reason = 3;
            S.status = -3;
            S.returned = j - 1;
            done_buf = S.cur;
          } else {
            if (dec == D_NEWMIN) {
              S.best0 = S.cur;
              S.best1 = nxt;
              S.best_j = j;
              S.xn_a = S.xn_prev;
              S.xn_b = xn;
            }
            S.xn_prev = xn;
            S.cur = nxt;
            if (j >= P.max_iter) {
              S.reason = 2;
              S.status = -4;
              S.returned = j;
              done_buf = nxt;
            }
          }
        }
        S.j = j;
        if (done_buf >= 0 && done_buf != nxt) {  // not the iterate the update wrote to the caller's X
          S.copy_buf = done_buf;
          done_buf = -1;
        }
        if (done_buf >= 0) {
          S.active = 0;
          if (tid == 0) {
            BInfo info;
            info.iters = j;
            info.returned = S.returned;
            info.reason = S.reason;
            info.status = S.status;
            info.alpha = S.alpha;
            info.dx_rel = S.dx_rel;
            info.sigma1_sq = S.sigma1_sq;
            P.info[b] = info;
          }
        }
        if (tid == 0) P.st[b] = S;
        __syncthreads();
      }
      if (P.trace && tid == 0) {
        if (t_item) busy += wall_clock64() - t_item;
        if (kTraceBusy + (int)blockIdx.x < kTraceCap) P.trace[kTraceBusy + blockIdx.x] = busy;
      }
      if (flowu && ph <= np) continue;
      if (!grid_sync(P.bar, G, nbar)) return;
      QP_STAMP();
    }
  }
#undef QP_STAMP
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
using BatchedLaunch = void (*)(const BParams&, int grid, hipStream_t);
using SyncLaunch = void (*)(const SParams&, int grid, hipStream_t);

template <class MM, int BM, int BN, int BK, int WM, int WN>
static void launch_batched(const BParams& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL((batched_kernel<MM, BM, BN, BK, WM, WN>), dim3(grid), dim3(64 * WM * WN), 0, s, P);
  QP_HIP(hipGetLastError());
}

template <class MM, int BM, int BN, int BK, int WM, int WN, int PER_CU = 2, bool FLOW = false>
static void launch_sync(const SParams& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL((batched_sync_kernel<MM, BM, BN, BK, WM, WN, PER_CU, FLOW>), dim3(grid), dim3(64 * WM * WN), 0, s,
                     P);
  QP_HIP(hipGetLastError());
}

template <class MM, int BM, int BN, int BK, int WM, int WN>
static int occupancy_of() {
  int nb = 0;
  QP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_kernel<MM, BM, BN, BK, WM, WN>, 64 * WM * WN, 0));
  return std::max(nb, 1);
}

template <class MM, int BM, int BN, int BK, int WM, int WN, int PER_CU = 2, bool FLOW = false>
static int occupancy_sync() {
  int nb = 0;
  QP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_sync_kernel<MM, BM, BN, BK, WM, WN, PER_CU, FLOW>,
                                                      64 * WM * WN, 0));
  return std::min(std::max(nb, 1), PER_CU);
}

// Queue kernels (one workgroup per matrix) and phase-synchronous kernels (all workgroups per product).
struct BatchedEntry {
  const char* name;
  BatchedLaunch fn;
  SyncLaunch sfn;
  int (*occ)();
  int bm, bn;
  bool flow;  // phase-synchronous kernel in its dataflow form (one grid barrier per update)
};

static const std::vector<BatchedEntry>& batched_table() {
  static const std::vector<BatchedEntry> t = {
      {"batched_f32_32x32x16_mfma16", launch_batched<MM16F, 32, 32, 16, 2, 2>, nullptr,
       occupancy_of<MM16F, 32, 32, 16, 2, 2>, 32, 32},
      {"batched_f32_64x64x16_mfma32", launch_batched<MM32F, 64, 64, 16, 2, 2>, nullptr,
       occupancy_of<MM32F, 64, 64, 16, 2, 2>, 64, 64},
      {"batched_f32_64x64x16_mfma16", launch_batched<MM16F, 64, 64, 16, 2, 2>, nullptr,
       occupancy_of<MM16F, 64, 64, 16, 2, 2>, 64, 64},
      {"batched_sync_f32_32x32x16_mfma16", nullptr, launch_sync<MM16F, 32, 32, 16, 2, 2>,
       occupancy_sync<MM16F, 32, 32, 16, 2, 2>, 32, 32},
      {"batched_sync_f32_64x64x16_mfma32", nullptr, launch_sync<MM32F, 64, 64, 16, 2, 2>,
       occupancy_sync<MM32F, 64, 64, 16, 2, 2>, 64, 64},
      {"batched_sync_f32_32x32x32_mfma16", nullptr, launch_sync<MM16F, 32, 32, 32, 2, 2>,
       occupancy_sync<MM16F, 32, 32, 32, 2, 2>, 32, 32},
      {"batched_flow_f32_32x32x32_mfma16", nullptr, launch_sync<MM16F, 32, 32, 32, 2, 2, 2, true>,
       occupancy_sync<MM16F, 32, 32, 32, 2, 2, 2, true>, 32, 32, true},
      {"batched_flow_f32_32x32x16_mfma16", nullptr, launch_sync<MM16F, 32, 32, 16, 2, 2, 2, true>,
       occupancy_sync<MM16F, 32, 32, 16, 2, 2, 2, true>, 32, 32, true},
  };
  return t;
}

int batched_num_configs() { return (int)batched_table().size(); }

const char* batched_config_name(int cfg) { return batched_table().at(cfg).name; }
bool batched_is_sync(int cfg) { return batched_table().at(cfg).sfn != nullptr; }

void batched_layout(std::vector<BDesc>& desc, int cfg, int64_t& pool, int64_t& part, int64_t& dwork) {
  const auto& ent = batched_table().at(cfg);
  auto up4 = [](int64_t x) { return (x + 3) / 4 * 4; };
  pool = part = dwork = 0;
  for (auto& d : desc) {
    const int64_t s = std::min(d.m, d.n);
    d.lds = up4(s);
    d.pss = s * d.lds;
    d.ldw = up4(d.m);
    d.psw = (int64_t)d.n * d.ldw;
    // the side product takes 16-byte loads of A: a copy unless its rows and planes are 16-byte aligned
    const bool aligned = ((d.lda | d.psa) & 3) == 0 && (reinterpret_cast<uintptr_t>(d.A) & 15) == 0;
    d.ldap = aligned ? 0 : up4(d.n);
    d.psap = (int64_t)d.m * d.ldap;
    d.off = pool;
    pool += 4 * (10 * d.pss + 5 * d.psw + d.psap);
    d.poff = part;
    part += 4 * (int64_t)((d.n + ent.bm - 1) / ent.bm) * ((d.m + ent.bn - 1) / ent.bn);  // 2 products x 2
    d.doff = dwork;
    dwork += 8 * (int64_t)std::max(d.m, d.n) + 8;
  }
}

__global__ void zero_int_kernel(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// timeout flag, barrier words and a status sentinel for every matrix (overwritten when it retires)
__global__ void sync_reset_kernel(unsigned int* bar, BInfo* info, int count, unsigned int* qctr, int qcap,
                                  unsigned int* done) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = i; k < BAR_WORDS; k += gridDim.x * blockDim.x) bar[k] = 0u;
  for (int k = i; k < qcap; k += gridDim.x * blockDim.x) qctr[k] = 0u;
  for (int b = i; b < count; b += gridDim.x * blockDim.x) {
    done[b] = 0u;
    info[b].iters = 0;
    info[b].returned = 0;
    info[b].reason = 0;
    info[b].status = -7;
    info[b].alpha = 0.0;
    info[b].dx_rel = 0.0;
    info[b].sigma1_sq = 0.0;
  }
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
  if (h_trace) (void)hipHostFree(h_trace);
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

// (Re)build the device buffers and the captured graph of a phase-synchronous configuration.
static void build_sync(BatchedState& st, const BKey& key, int64_t pool_cap, int64_t part_cap, int64_t dw_cap) {
  st.~BatchedState();
  new (&st) BatchedState();
  st.key = key;
  st.pool_cap = pool_cap;
  st.part_cap = part_cap;
  st.dw_cap = dw_cap;
  const int count = key.count;
  const auto& ent = batched_table().at(key.cfg);
  int dev = 0, cus = 0;
  QP_HIP(hipGetDevice(&dev));
  QP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // every workgroup must be resident for the grid barrier: at most the occupancy per compute unit
  st.grid = std::max(1, cus * ent.occ());
  QP_HIP(hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking));
  QP_HIP(hipEventCreateWithFlags(&st.ev0, hipEventDisableTiming));
  QP_HIP(hipEventCreateWithFlags(&st.ev1, hipEventDisableTiming));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_desc), sizeof(BDesc) * count, hipHostMallocDefault));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_info), sizeof(BInfo) * count, hipHostMallocDefault));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_order), sizeof(int) * 4, hipHostMallocDefault));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_alpha), sizeof(double) * count, hipHostMallocDefault));
  BDesc* d_desc = static_cast<BDesc*>(dev_alloc(st, sizeof(BDesc) * count));
  BInfo* d_info = static_cast<BInfo*>(dev_alloc(st, sizeof(BInfo) * count));
  LState* d_st = static_cast<LState*>(dev_alloc(st, sizeof(LState) * count));
  unsigned int* d_bar = static_cast<unsigned int*>(dev_alloc(st, sizeof(unsigned int) * BAR_WORDS));
  // one item counter per phase: (max_iter + 2) passes of at most 32 phases
  const int qcap = (key.max_iter + 2) * 32;
  unsigned int* d_qctr = static_cast<unsigned int*>(dev_alloc(st, sizeof(unsigned int) * (size_t)qcap));
  unsigned int* d_done = static_cast<unsigned int*>(dev_alloc(st, sizeof(unsigned int) * (size_t)count));
  double* d_alpha = static_cast<double*>(dev_alloc(st, sizeof(double) * count));
  float* pool = static_cast<float*>(dev_alloc(st, sizeof(float) * (size_t)pool_cap));
  double* partial = static_cast<double*>(dev_alloc(st, sizeof(double) * (size_t)part_cap));
  double* dwork = static_cast<double*>(dev_alloc(st, sizeof(double) * (size_t)dw_cap));
  unsigned long long* trace = static_cast<unsigned long long*>(dev_alloc(st, sizeof(unsigned long long) * kTraceCap));
  QP_HIP(hipHostMalloc(reinterpret_cast<void**>(&st.h_trace), sizeof(unsigned long long) * kTraceCap,
                       hipHostMallocDefault));

  SParams P;
  P.desc = d_desc;
  P.info = d_info;
  P.st = d_st;
  P.count = count;
  P.pool = pool;
  P.partial = partial;
  P.dwork = dwork;
  P.bar = d_bar;
  P.alpha = d_alpha;
  P.method = key.method;
  P.stop = key.stop;
  P.max_iter = key.max_iter;
  P.tol = key.tol;
  P.scaling = key.scaling;
  P.power_steps = key.power_steps;
  P.seed = key.seed;
  P.k = make_coef();
  P.trace = trace;
  P.trace_cap = kTraceCap;
  P.qctr = d_qctr;
  P.qctr_cap = qcap;
  P.dyn = key.dyn;
  P.done = d_done;

  hipStream_t s = st.stream;
  QP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  QP_HIP(hipMemcpyAsync(d_desc, st.h_desc, sizeof(BDesc) * count, hipMemcpyHostToDevice, s));
  QP_HIP(hipMemcpyAsync(d_alpha, st.h_alpha, sizeof(double) * count, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(sync_reset_kernel, dim3((count + 255) / 256 + 1), dim3(256), 0, s, d_bar, d_info, count, d_qctr,
                     qcap, d_done);
  ent.sfn(P, st.grid, s);
  QP_HIP(hipMemcpyAsync(st.h_info, d_info, sizeof(BInfo) * count, hipMemcpyDeviceToHost, s));
  QP_HIP(hipMemcpyAsync(st.h_order, d_bar, sizeof(unsigned int) * 4, hipMemcpyDeviceToHost, s));
  QP_HIP(hipMemcpyAsync(st.h_trace, trace, sizeof(unsigned long long) * kTraceCap, hipMemcpyDeviceToHost, s));
  QP_HIP(hipStreamEndCapture(s, &st.graph));
  QP_HIP(hipGraphInstantiate(&st.exec, st.graph, nullptr, nullptr, 0));
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

void run_batched(BatchedState& st, const BKey& key, const std::vector<BDesc>& desc_in, const std::vector<int>& order,
                 const std::vector<double>& alphas, std::vector<BInfo>& infos, hipStream_t caller, bool verbose) {
  const int count = key.count;
  const bool sync = batched_is_sync(key.cfg);
  std::vector<BDesc> desc = desc_in;
  if (sync) {
    if (count > SYNC_MAX) throw Error(-1, "phase-synchronous batched solves take at most 2048 matrices");
    int64_t pool = 0, part = 0, dw = 0;
    batched_layout(desc, key.cfg, pool, part, dw);
    if (!st.exec || !(st.key == key) || pool > st.pool_cap || part > st.part_cap || dw > st.dw_cap)
      build_sync(st, key, pool + pool / 4 + 64, part + part / 4 + 64, dw + dw / 4 + 64);
  } else if (!st.exec || !(st.key == key) || st.pool_cap != 0) {
    build(st, key, caller);
  }
  std::memcpy(st.h_desc, desc.data(), sizeof(BDesc) * count);
  if (!sync) std::memcpy(st.h_order, order.data(), sizeof(int) * count);
  for (int b = 0; b < count; ++b) st.h_alpha[b] = b < (int)alphas.size() ? alphas[b] : 0.0;
  // order the graph after the caller's stream, and the caller after the graph
  QP_HIP(hipEventRecord(st.ev0, caller));
  QP_HIP(hipStreamWaitEvent(st.stream, st.ev0, 0));
  QP_HIP(hipGraphLaunch(st.exec, st.stream));
  QP_HIP(hipEventRecord(st.ev1, st.stream));
  QP_HIP(hipStreamWaitEvent(caller, st.ev1, 0));
  QP_HIP(hipStreamSynchronize(st.stream));
  infos.assign(st.h_info, st.h_info + count);
  if (sync && verbose) {
    // phase durations from the barrier stamps (100 MHz wall clock): per update, the np product phases
    // and the controller phase
    const unsigned long long* t = st.h_trace;
    const int np = key.method == 0 ? 2 : key.method == 2 ? 6 : 7;
    const bool flow = batched_table().at(key.cfg).flow;  // then the updates' stamp counts differ
    fprintf(stderr, "[qpinv] batched set-up %.1f us\n", (double)(t[1] - t[0]) * 1e-2);
    {  // per-matrix set-up durations (stamped by the workgroup that did it)
      double mx = 0.0, sum = 0.0;
      int arg = 0;
      for (int b = 0; b < count && kTraceSetup + b < kTraceBusy; ++b) {
        const double v = (double)t[kTraceSetup + b] * 1e-2;
        sum += v;
        if (v > mx) {
          mx = v;
          arg = b;
        }
      }
      fprintf(stderr, "[qpinv] batched per-matrix set-up: mean %.1f us, max %.1f us (matrix %d, %d x %d)\n",
              sum / std::max(count, 1), mx, arg, desc[arg].m, desc[arg].n);
    }
    int k = 2;
    while (k < kTraceSetup && t[k] > t[k - 1] && t[k] - t[k - 1] < 100000000ull) {
      if (flow) {
        if (k == 2) fprintf(stderr, "[qpinv] batched barrier intervals (us):");
        fprintf(stderr, " %.1f", (double)(t[k] - t[k - 1]) * 1e-2);
      } else {
        if ((k - 2) % (np + 1) == 0) fprintf(stderr, "[qpinv] batched update %d:", (k - 2) / (np + 1) + 1);
        fprintf(stderr, " %.1f", (double)(t[k] - t[k - 1]) * 1e-2);
        if ((k - 2) % (np + 1) == np) fprintf(stderr, " us\n");
      }
      ++k;
    }
    fprintf(stderr, "\n");
    {  // share of the update time the workgroups spent inside work items
      const double upd = (double)(t[k - 1] - t[1]) * 1e-2;
      double sum = 0.0, mx = 0.0;
      const int G = st.grid;
      for (int g = 0; g < G && kTraceBusy + g < kTraceCap; ++g) {
        const double v = (double)t[kTraceBusy + g] * 1e-2;
        sum += v;
        mx = std::max(mx, v);
      }
      fprintf(stderr, "[qpinv] batched updates %.1f us; workgroups inside items: mean %.1f us (%.1f%%), max %.1f us\n",
              upd, sum / std::max(G, 1), upd > 0 ? 100.0 * sum / std::max(G, 1) / upd : 0.0, mx);
    }
  }
  if (sync && reinterpret_cast<const unsigned int*>(st.h_order)[2] != 0u)
    throw Error(-7, "batched solve: a grid barrier wait expired (workgroups not co-resident?)");
}

}  // namespace qp

// Single solves of small matrices (at most 128 per side) in ONE kernel launch.
//
// A solve of a 64 x 48 matrix is a chain of about thirty 48 x 48 products, each a few microseconds of MFMA
// work: launched one by one, with the stop rule read on the host after every update, launch gaps and
// synchronisations take most of the time.  Here one persistent launch runs the whole solve: workgroup 0
// computes ||A||_F, the finiteness check and the power iteration, the grid forms X_0 = alpha A^H, and then
// every product of every update is a phase whose items are 16 x 16 output blocks (all four planes), dealt to
// the workgroups, which meet at a bounded grid barrier after each phase.  Within a block the 16 waves split
// the four output planes and four slices of K (each lane's partial sums meet in LDS), so a product of
// K = 64 costs each wave 16 MFMAs instead of the 256 one wave would issue alone.  The per-element epilogue
// is the standalone product kernel's (identity shifts, polynomial combinations, change norms).
//
// The products and epilogues of an update are the chain of the regular path (a program the host builds
// per method and side).  After the update phase every workgroup sums the change norms of the update in the
// same fixed order and takes the same stop decision, so no further barrier is needed.  The E1 rule reuses
// the next update's residual: on the left side A R = A - A X A (right side R A), one extra product in the
// phase that forms R^2, so ||A X_j A - A||_F for the iterate X_j just made is known after the next update's
// second phase, and the solve stops there, returning X_j, when it meets the tolerance.
//
// Every wait is bounded: a workgroup that waits too long raises a flag, all leave at the next barrier,
// and the host reports ETIMEOUT.  The grid is at most the number of output blocks of the largest phase
// (<= 128), one workgroup per compute unit, so all of it is resident.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "aux.hpp"
#include "controller.hpp"
#include "qgemm_kern.hpp"
#include "solver.hpp"

namespace qp {
namespace {

constexpr int SM_MAXD = 128;
constexpr int SM_KSPLIT = 2;
constexpr int SM_THREADS = 256 * SM_KSPLIT;
constexpr int SM_MAXG = 128;
constexpr long long SM_SPIN_MAX = 1ll << 22;  // barrier polls before the wait is abandoned

// buffers of the solve: A, the two iterates (current / next resolved per update), 8 side-by-side, and the
// E1 product A R (left) or R A (right), m x n
enum : int { B_A = 0, B_XC = 1, B_XN = 2, B_SQ = 3, B_E = 11, B_N = 12 };

struct SmView {
  void* p;
  int64_t ld, ps;
  int rows, cols;
};

struct SmProd {
  int a, b;               // operand buffers
  int nout, nin, ref;     // epilogue shape (as Epilogue)
  int reduce;             // 0 none, 1 update change norms, 2 sum of squares of the output (E1)
  int out[3], in[3];
  double ca[3], cg[3], cb[3][3];
};

struct SmProgram {
  int nphase;        // phases of one update; the last forms X_{j+1}
  int e1_phase;      // phase whose second product is the E1 product (-1: none)
  int nprod[8];
  SmProd prod[8][2];
};

template <class T>
struct SmParams {
  SmView buf[B_N];       // B_XC / B_XN hold iterate buffers 0 / 1
  T* xout;               // the caller's X (n x m), written directly when xout_direct
  int64_t ldx, psx;
  int xout_direct;
  SmProgram prog;
  int m, n;
  int scaling, power_steps;
  unsigned long long seed;
  double alpha_given, mu;
  int stop, max_iter;
  double tol;
  double* partial;       // [2][2][SM_MAXG * 2]: per item reduction terms (slot by phase kind)
  double* state;         // result record (see SmState)
  unsigned int* bar;     // [0] arrivals, [1] generation, [2] give-up flag
  unsigned long long* trace;  // optional (option verbose): workgroup 0 stamps wall_clock64() after each barrier
  int trace_cap;
};

// result record, doubles
enum : int {
  S_STATUS = 0, S_ITERS, S_RETURNED, S_REASON, S_ALPHA, S_S1SQ, S_NORMA2, S_DXREL, S_E1, S_RETBUF, S_NONFINITE,
  S_COUNT
};

__device__ __forceinline__ uint64_t sm_splitmix64(uint64_t counter, uint64_t seed) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// sign of a_q b_{p^q} in plane p of a Hamilton product (p^q: the b plane it multiplies)
__device__ __forceinline__ double qsign(int p, int q) {
  if (q == 0) return 1.0;
  if (q == 1) return (p == 0 || p == 2) ? -1.0 : 1.0;
  if (q == 2) return (p == 0 || p == 3) ? -1.0 : 1.0;
  return (p == 0 || p == 1) ? -1.0 : 1.0;
}

// Grid barrier (counter and generation in device memory); false once any workgroup has abandoned a wait.
__device__ bool sm_sync(unsigned int* bar, unsigned int nblocks) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    // the generation is read before arriving; the arrival releases this workgroup's writes (and, for the
    // last to arrive, acquires everyone's); waiters poll relaxed and acquire once when the generation moves
    const unsigned int gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned int arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == nblocks) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > SM_SPIN_MAX) {
          __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ok = 0;
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// workgroup sum of a double, fixed order (every thread gets it)
__device__ __forceinline__ double sm_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  return t;
}

template <class T>
__device__ __forceinline__ SmView resolve(const SmParams<T>* P, int b, int cur) {
  if (b == B_XC) return P->buf[1 + cur];
  if (b == B_XN) return P->buf[2 - cur];
  return P->buf[b];
}

// Workgroup-uniform values to scalar registers (the per-item product parameters stay out of the vector budget).
__device__ __forceinline__ int su(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t su(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ float su(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double su(double v) { return __longlong_as_double(su((int64_t)__double_as_longlong(v))); }
template <class T>
__device__ __forceinline__ T* su(T* p) {
  return reinterpret_cast<T*>(su((int64_t)reinterpret_cast<uintptr_t>(p)));
}

template <class T>
__device__ __forceinline__ void make_uniform(GemmParams<T>& G) {
  G.A = su(G.A);
  G.lda = su(G.lda);
  G.psa = su(G.psa);
  G.B = su(G.B);
  G.ldb = su(G.ldb);
  G.psb = su(G.psb);
  G.M = su(G.M);
  G.N = su(G.N);
  G.K = su(G.K);
  G.tiles_m = su(G.tiles_m);
  G.tiles_n = su(G.tiles_n);
  G.nout = su(G.nout);
  G.nin = su(G.nin);
  G.ref = su(G.ref);
  G.reduce = su(G.reduce);
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    G.out[t] = su(G.out[t]);
    G.ldo[t] = su(G.ldo[t]);
    G.pso[t] = su(G.pso[t]);
    G.in[t] = su(G.in[t]);
    G.ldi[t] = su(G.ldi[t]);
    G.psi[t] = su(G.psi[t]);
    G.ca[t] = su(G.ca[t]);
    G.cg[t] = su(G.cg[t]);
#pragma unroll
    for (int u = 0; u < 3; ++u) G.cb[t][u] = su(G.cb[t][u]);
  }
}

template <class T>
__device__ __forceinline__ GemmParams<T> make_gemm(const SmParams<T>* P, const SmProd& d, int cur) {
  GemmParams<T> G{};
  const SmView a = resolve(P, d.a, cur), b = resolve(P, d.b, cur);
  G.A = static_cast<const T*>(a.p);
  G.lda = a.ld;
  G.psa = a.ps;
  G.B = static_cast<const T*>(b.p);
  G.ldb = b.ld;
  G.psb = b.ps;
  G.M = a.rows;
  G.N = b.cols;
  G.K = a.cols;
  G.tiles_m = (G.M + 15) / 16;
  G.tiles_n = (G.N + 15) / 16;
  G.nout = d.nout;
  G.nin = d.nin;
  G.ref = d.ref;
  for (int t = 0; t < 3; ++t) {
    const SmView o = resolve(P, t < d.nout ? d.out[t] : d.a, cur);
    const SmView in = resolve(P, t < d.nin ? d.in[t] : d.a, cur);
    G.out[t] = t < d.nout ? static_cast<T*>(o.p) : nullptr;
    G.ldo[t] = o.ld;
    G.pso[t] = o.ps;
    G.in[t] = t < d.nin ? static_cast<const T*>(in.p) : nullptr;
    G.ldi[t] = in.ld;
    G.psi[t] = in.ps;
    G.ca[t] = (T)d.ca[t];
    G.cg[t] = (T)d.cg[t];
    for (int u = 0; u < 3; ++u) G.cb[t][u] = (T)d.cb[t][u];
  }
  G.reduce = d.reduce != 0;
  make_uniform(G);
  return G;
}

// One 16 x 16 output block (all four planes) of C = A B with the epilogue.  The block's operands are staged
// in LDS SM_KB deep in k, every thread loading two elements of each (one memory latency per round): A as
// [plane][row][k], B as [plane][k][column], both padded by one element.  Wave w then takes output plane w % 4
// and the k chunks (of 4) with index = w / 4 modulo SM_KSPLIT; the slices' partial sums meet in LDS (`red`,
// which reuses the staging area), and the first slice's waves run the epilogue.  The reduction terms are
// added to s_d, s_x.
constexpr int SM_KB = 64;  // k staged per round (products of K <= 64 take one round)
template <class T>
constexpr int sm_stage_elems() {
  return 4 * 16 * (SM_KB + 1) + 4 * SM_KB * 17;
}

template <class T, class MM>
__device__ void sm_block(const GemmParams<T>& G, int tm, int tn, T* stage, typename MM::Acc* red, double& s_d,
                         double& s_x) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int p = w & 3, ks = w >> 2;
  const int rb = tm * 16, cb = tn * 16;
  T* const As = stage;
  T* const Bs = stage + 4 * 16 * (SM_KB + 1);
  typename MM::Acc acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = T(0);
  const T s1 = (T)qsign(p, 1), s2 = (T)qsign(p, 2), s3 = (T)qsign(p, 3);
  // the epilogue's inputs do not depend on the product: their loads go out with the operands'
  T inv[4][3];
  if (ks == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) epilogue_inputs(G, p, rb + MM::crow(lane, r), cb + MM::ccol(lane), inv[r]);
  }
  constexpr int NU = 4 * 16 * SM_KB / SM_THREADS;  // staged elements of each operand per thread, at most
  for (int k0 = 0; k0 < G.K; k0 += SM_KB) {
    const int kr = G.K - k0 < SM_KB ? G.K - k0 : SM_KB;  // k of this round
    const int kr4 = (kr + 3) & ~3;
    const int lim = 4 * 16 * kr4;
    // every load is issued before the first LDS store (one memory latency per round); addresses are clamped
    // into the operands and the values outside them replaced by zeros
    T va[NU], vb[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + u * SM_THREADS;
      // A: k fastest (rows of A are contiguous in k); B: columns fastest
      const int qa = e / (16 * kr4), ra = (e / kr4) % 16, kka = e % kr4;
      const int row = rb + ra, ka = k0 + kka;
      const bool oka = e < lim && row < G.M && ka < G.K;
      const int qb = e / (kr4 * 16), kkb = (e / 16) % kr4, cc = e % 16;
      const int col = cb + cc, kb = k0 + kkb;
      const bool okb = e < lim && kb < G.K && col < G.N;
      va[u] = gload(G.A, (oka ? qa : 0) * G.psa + (int64_t)(oka ? row : 0) * G.lda + (oka ? ka : 0));
      vb[u] = gload(G.B, (okb ? qb : 0) * G.psb + (int64_t)(okb ? kb : 0) * G.ldb + (okb ? col : 0));
      va[u] = oka ? va[u] : T(0);
      vb[u] = okb ? vb[u] : T(0);
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + u * SM_THREADS;
      if (e < lim) {
        As[((e / (16 * kr4)) * 16 + (e / kr4) % 16) * (SM_KB + 1) + e % kr4] = va[u];
        Bs[((e / (kr4 * 16)) * SM_KB + (e / 16) % kr4) * 17 + e % 16] = vb[u];
      }
    }
    __syncthreads();
    const int r16 = lane & 15, kl = lane >> 4;
    for (int kc = ks; kc < kr4 / 4; kc += SM_KSPLIT) {
      const int kk = kc * 4 + kl;
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[(q * 16 + r16) * (SM_KB + 1) + kk];
        b[q] = Bs[((p ^ q) * SM_KB + kk) * 17 + r16];
      }
      acc = MM::mma(a[0], b[0], acc);
      acc = MM::mma(s1 * a[1], b[1], acc);
      acc = MM::mma(s2 * a[2], b[2], acc);
      acc = MM::mma(s3 * a[3], b[3], acc);
    }
    __syncthreads();
  }
  // slices 1..3 hand their sums to slice 0 (red: [SM_KSPLIT - 1][4 planes][64 lanes])
  if (ks > 0) red[((ks - 1) * 4 + p) * 64 + lane] = acc;
  __syncthreads();
  if (ks == 0) {
#pragma unroll
    for (int s = 1; s < SM_KSPLIT; ++s) {
      const typename MM::Acc o = red[((s - 1) * 4 + p) * 64 + lane];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] += o[r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) epilogue_apply(G, p, rb + MM::crow(lane, r), cb + MM::ccol(lane), acc[r], inv[r], s_d, s_x);
  }
  __syncthreads();  // the staging area is reused by the next block
}

// w = A v (adj = false; v: 4 n, w: 4 m) or w = A^H v (adj = true; v: 4 m, w: 4 n), planes [p][i], in LDS;
// part holds the column-chunk partial sums.  Sums over fixed chunks in a fixed order.
template <class T>
__device__ void sm_gemv(const T* a, int64_t lda, int64_t psa, int m, int n, bool adj, const double* v, double* w,
                        double* part) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int rows = adj ? n : m, cols = adj ? m : n;
  const int chunks = nt / rows;  // rows <= 128 -> at least 4
  if (tid < rows * chunks) {
    const int i = tid % rows, c = tid / rows;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = c; j < cols; j += chunks) {
      // element (i, j) of A or of A^H (= conj of A's (j, i))
      const int64_t off = adj ? (int64_t)j * lda + i : (int64_t)i * lda + j;
      double aq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) aq[q] = (double)a[q * psa + off];
      if (adj) {
        aq[1] = -aq[1];
        aq[2] = -aq[2];
        aq[3] = -aq[3];
      }
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
#pragma unroll
        for (int q = 0; q < 4; ++q) s[pl] += qsign(pl, q) * aq[q] * v[(pl ^ q) * cols + j];
    }
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) part[(c * 4 + pl) * rows + i] = s[pl];
  }
  __syncthreads();
  if (tid < 4 * rows) {
    const int pl = tid / rows, i = tid % rows;
    double t = 0.0;
    for (int c = 0; c < chunks; ++c) t += part[(c * 4 + pl) * rows + i];
    w[pl * rows + i] = t;
  }
  __syncthreads();
}

template <class T, class MM>
__global__ void __launch_bounds__(SM_THREADS) small_solve_kernel(const SmParams<T>* __restrict__ Pg) {
  // one LDS area serves the K-slice exchange of the products ((SM_KSPLIT - 1) x 4 planes x 64 lanes of
  // accumulators) and the power iteration's chunk sums (chunks x 4 planes x rows <= 4 x threads doubles)
  // one LDS area: the operand staging of a product (whole K), the K-slice exchange after it, and in the
  // set-up the power iteration's chunk sums followed by a copy of A when A fits
  constexpr int RED_BYTES = (SM_KSPLIT - 1) * 4 * 64 * (int)sizeof(typename MM::Acc);
  constexpr int PART_BYTES = 4 * SM_THREADS * (int)sizeof(double);
  constexpr int STAGE_BYTES = sm_stage_elems<T>() * (int)sizeof(T);
  constexpr int SETUP_BYTES = 120 * 1024;  // chunk sums + a copy of A of up to 104 KB
  constexpr int LDS_BYTES0 = STAGE_BYTES > RED_BYTES ? STAGE_BYTES : RED_BYTES;
  constexpr int LDS_BYTES = LDS_BYTES0 > SETUP_BYTES ? LDS_BYTES0 : SETUP_BYTES;
  static_assert(LDS_BYTES >= PART_BYTES, "set-up scratch fits");
  __shared__ __attribute__((aligned(16))) unsigned char lds[LDS_BYTES];
  typename MM::Acc* const red = reinterpret_cast<typename MM::Acc*>(lds);
  double* const part = reinterpret_cast<double*>(lds);
  T* const stage = reinterpret_cast<T*>(lds);
  T* const acopy = reinterpret_cast<T*>(lds + PART_BYTES);
  constexpr int ACOPY_ELEMS = (LDS_BYTES - PART_BYTES) / (int)sizeof(T);
  __shared__ double sh[32];
  __shared__ double vs[4 * SM_MAXD], wsv[4 * SM_MAXD];
  // the parameter block, read once from device memory (phases index it by product and buffer)
  __shared__ __attribute__((aligned(16))) unsigned int pcopy[(sizeof(SmParams<T>) + 3) / 4];
  {
    const unsigned int* src = reinterpret_cast<const unsigned int*>(Pg);
    for (int i = threadIdx.x; i < (int)((sizeof(SmParams<T>) + 3) / 4); i += blockDim.x) pcopy[i] = src[i];
    __syncthreads();
  }
  const SmParams<T>* const P = reinterpret_cast<const SmParams<T>*>(pcopy);
  const int tid = threadIdx.x;
  const unsigned int G = gridDim.x;
  int nstamp = 0;
  auto stamp = [&]() {
    if (P->trace && blockIdx.x == 0 && tid == 0 && nstamp < P->trace_cap) P->trace[nstamp] = wall_clock64();
    ++nstamp;
  };
  stamp();
  const int m = P->m, n = P->n;
  const SmView A = P->buf[B_A];
  const T* a = static_cast<const T*>(A.p);

  // ---------------------------------------------------------------- set-up (workgroup 0)
  if (blockIdx.x == 0) {
    double fro = 0.0, bad = 0.0;
    for (int e = tid; e < 4 * m * n; e += blockDim.x) {
      const int pl = e / (m * n), r = (e / n) % m, c = e % n;
      const double x = (double)gload(a, pl * A.ps + (int64_t)r * A.ld + c);
      if (!__builtin_isfinite(x)) bad += 1.0;
      fro += x * x;
    }
    fro = sm_sum(fro, sh);
    bad = sm_sum(bad, sh);
    double alpha = 0.0, s1sq = 0.0;
    if (bad == 0.0 && fro > 0.0) {
      if (P->scaling == QPINV_ALPHA_POWER) {
        // A into LDS when it fits (every power step reads all of it twice)
        const bool in_lds = 4 * m * n <= ACOPY_ELEMS;
        if (in_lds)
          for (int e = tid; e < 4 * m * n; e += blockDim.x) {
            const int pl = e / (m * n), r = (e / n) % m, c = e % n;
            acopy[e] = gload(a, pl * A.ps + (int64_t)r * A.ld + c);
          }
        const T* const ap = in_lds ? acopy : a;
        const int64_t ald = in_lds ? n : A.ld, aps = in_lds ? (int64_t)m * n : A.ps;
        for (int e = tid; e < 4 * n; e += blockDim.x)
          vs[e] = (double)(sm_splitmix64((uint64_t)e, P->seed) >> 11) * 0x1p-52 - 1.0;
        __syncthreads();
        for (int it = 0; it < P->power_steps; ++it) {
          double vv = 0.0;
          for (int e = tid; e < 4 * n; e += blockDim.x) vv += vs[e] * vs[e];
          vv = sm_sum(vv, sh);
          const double inv = 1.0 / sqrt(vv);
          for (int e = tid; e < 4 * n; e += blockDim.x) vs[e] *= inv;
          __syncthreads();
          sm_gemv<T>(ap, ald, aps, m, n, false, vs, wsv, part);
          double ww = 0.0;
          for (int e = tid; e < 4 * m; e += blockDim.x) ww += wsv[e] * wsv[e];
          s1sq = sm_sum(ww, sh);
          sm_gemv<T>(ap, ald, aps, m, n, true, wsv, vs, part);
        }
        alpha = (P->mu > 0.0 ? P->mu : 1.0) / s1sq;
      } else if (P->scaling == QPINV_ALPHA_FROB) {
        alpha = 1.0 / fro;
      } else {
        alpha = P->alpha_given;
      }
    }
    if (tid == 0) {
      P->state[S_NONFINITE] = bad;
      P->state[S_NORMA2] = fro;
      P->state[S_ALPHA] = alpha;
      P->state[S_S1SQ] = s1sq;
    }
  }
  if (!sm_sync(P->bar, G)) return;
  stamp();
  const double bad = __hip_atomic_load(&P->state[S_NONFINITE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double fro = __hip_atomic_load(&P->state[S_NORMA2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double alpha = __hip_atomic_load(&P->state[S_ALPHA], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (bad != 0.0) {
    if (blockIdx.x == 0 && tid == 0) P->state[S_STATUS] = QPINV_ENONFINITE;
    return;
  }
  const double normA = sqrt(fro);
  const int gtid = blockIdx.x * blockDim.x + tid, gthreads = G * blockDim.x;

  // ---------------------------------------------------------------- X_0 = alpha A^H into iterate 0
  {
    const SmView X0 = P->buf[1];
    T* x = static_cast<T*>(X0.p);
    for (int e = gtid; e < 4 * m * n; e += gthreads) {
      const int pl = e / (m * n), r = (e / m) % n, c = e % m;  // X0 element (r, c) = conj(A(c, r))
      const T v = gload(a, pl * A.ps + (int64_t)c * A.ld + r);
      gstore(x, pl * X0.ps + (int64_t)r * X0.ld + c, (T)(alpha * (double)(pl == 0 ? v : -v)));
    }
  }
  if (!sm_sync(P->bar, G)) return;
  stamp();

  // ---------------------------------------------------------------- updates
  StopController ctl(P->stop, P->tol);
  const bool e1 = P->stop == STOP_E1_REL;
  int cur = 0, j = 0;
  int status = QPINV_OK, reason = QPINV_REASON_TOL, ret_buf = 0, ret_j = 0;
  double dx_rel = 0.0, e1_rel = -1.0;
  bool done = normA == 0.0;  // A = 0: X_0 = 0 is the pseudoinverse
  while (!done) {
    for (int ph = 0; ph < P->prog.nphase && !done; ++ph) {
      const int np = P->prog.nprod[ph];
      // output blocks of the phase's products (X_0's E1 is never needed)
      int tiles[2] = {0, 0};
      for (int q = 0; q < 2; ++q) {
        if (q >= np || (q == 1 && ph == P->prog.e1_phase && j == 0)) continue;
        const SmProd& d = P->prog.prod[ph][q];
        const SmView a = resolve(P, d.a, cur), b = resolve(P, d.b, cur);
        tiles[q] = ((a.rows + 15) / 16) * ((b.cols + 15) / 16);
      }
      const int total = tiles[0] + tiles[1];
      for (int item = blockIdx.x; item < total; item += G) {
        const int q = item < tiles[0] ? 0 : 1;
        const int t = item - (q ? tiles[0] : 0);
        const GemmParams<T> gq = make_gemm(P, P->prog.prod[ph][q], cur);
        double s_d = 0.0, s_x = 0.0;
        sm_block<T, MM>(gq, t / gq.tiles_n, t % gq.tiles_n, stage, red, s_d, s_x);
        const int kind = P->prog.prod[ph][q].reduce;
        if (kind) {
          s_d = sm_sum(s_d, sh);
          s_x = sm_sum(s_x, sh);
          if (tid == 0) {
            double* slot = P->partial + (kind - 1) * 2 * 2 * SM_MAXG;
            slot[2 * t] = s_d;
            slot[2 * t + 1] = s_x;
          }
        }
      }
      if (!sm_sync(P->bar, G)) return;
  stamp();
      if (e1 && ph == P->prog.e1_phase && j >= 1) {
        // ||A X_j A - A||_F / ||A||_F from the tiles of the E1 product, summed in tile order
        double s = 0.0;
        for (int t = 0; t < tiles[1]; ++t) s += P->partial[2 * 2 * SM_MAXG + 2 * t + 1];
        e1_rel = sqrt(s) / normA;
        const int dec = ctl.update(j, 0.0, 1.0, e1_rel);
        if (dec == D_DIVERGED) {
          status = QPINV_EDIVERGED;
          reason = QPINV_REASON_DIVERGED;
          done = true;
        } else if (dec == D_TOL) {
          done = true;
        } else if (j >= P->max_iter) {
          status = QPINV_ENOTCONVERGED;
          reason = QPINV_REASON_MAX_ITER;
          done = true;
        }
        if (done) {
          ret_buf = cur;
          ret_j = j;
        }
      }
      if (done || ph != P->prog.nphase - 1) continue;
      // the update X_{j+1} = X_nxt is formed: change norms in tile order, then the stop rule
      const int tu = P->prog.prod[ph][0].reduce == 1 ? tiles[0] : 0;
      double d2 = 0.0, x2 = 0.0;
      for (int t = 0; t < tu; ++t) {
        d2 += P->partial[2 * t];
        x2 += P->partial[2 * t + 1];
      }
      const double d_abs = sqrt(fmax(0.0, d2)), xn = sqrt(fmax(0.0, x2));
      ++j;
      dx_rel = xn > 0.0 ? d_abs / xn : 0.0;
      const bool diverged = !__builtin_isfinite(d_abs) || !__builtin_isfinite(xn) || xn * normA > 1e20;
      if (diverged) {
        status = QPINV_EDIVERGED;
        reason = QPINV_REASON_DIVERGED;
        ret_buf = __builtin_isfinite(xn) ? 1 - cur : cur;
        ret_j = __builtin_isfinite(xn) ? j : j - 1;
        done = true;
      } else if (!e1) {
        const int dec = ctl.update(j, d_abs, xn, -1.0);
        if (dec == D_TOL) {
          ret_buf = 1 - cur;
          ret_j = j;
          done = true;
        } else if (j >= P->max_iter) {
          status = QPINV_ENOTCONVERGED;
          reason = QPINV_REASON_MAX_ITER;
          ret_buf = 1 - cur;
          ret_j = j;
          done = true;
        }
      }
      cur = 1 - cur;
      if (done) break;
    }
  }
  if (normA == 0.0) ret_buf = 0;  // X_0 = 0

  // ---------------------------------------------------------------- result
  if (P->xout_direct) {
    const SmView Xr = P->buf[1 + ret_buf];
    const T* x = static_cast<const T*>(Xr.p);
    for (int e = gtid; e < 4 * m * n; e += gthreads) {
      const int pl = e / (m * n), r = (e / m) % n, c = e % m;
      gstore(P->xout, pl * P->psx + (int64_t)r * P->ldx + c, gload(x, pl * Xr.ps + (int64_t)r * Xr.ld + c));
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    P->state[S_STATUS] = status;
    P->state[S_ITERS] = j;
    P->state[S_RETURNED] = ret_j;
    P->state[S_REASON] = reason;
    P->state[S_DXREL] = dx_rel;
    P->state[S_E1] = e1_rel;
    P->state[S_RETBUF] = ret_buf;
  }
}

// ------------------------------------------------------------------------------------------------
// host: the update program (the regular chain's products and epilogues), eligibility, launch
// ------------------------------------------------------------------------------------------------
const double kS5 = std::sqrt(5.0);
const double kBeta1 = 0.5 * (1.0 + kS5), kBeta2 = 0.5 * (1.0 - kS5);
const double kS93 = std::sqrt(93.0), kRt = std::sqrt(27.0 - 2.0 * kS93);
const double kD1 = 0.25 * (1.0 + kRt), kD2 = 0.25 * (1.0 - kRt), kD3 = (5.0 * kS93 - 93.0) / 496.0;
const double kE1 = (-93.0 - 5.0 * kS93) / 496.0, kE2 = -0.25 * kS93, kC1 = 3.0 / 8.0, kC2 = 321.0 / 1984.0;

SmProd prod(int a, int b, int out, double ca = 1.0, double cg = 0.0) {
  SmProd d;
  std::memset(&d, 0, sizeof(d));
  d.a = a;
  d.b = b;
  d.nout = 1;
  d.out[0] = out;
  d.ca[0] = ca;
  d.cg[0] = cg;
  d.ref = 3;
  return d;
}

int sq(int k) { return B_SQ + k; }

// Products of one update of `method` on `side` (left: R = I - X A, X+ = T X; right: R = I - A X, X+ = X T).
SmProgram build_program(int method, bool left, bool e1) {
  SmProgram g;
  std::memset(&g, 0, sizeof(g));
  g.e1_phase = -1;
  auto side_prod = [&](int out, double ca, double cg) { return left ? prod(B_XC, B_A, out, ca, cg) : prod(B_A, B_XC, out, ca, cg); };
  auto update = [&](int T) {
    SmProd d = left ? prod(T, B_XC, B_XN) : prod(B_XC, T, B_XN);
    d.nin = 1;
    d.in[0] = B_XC;
    d.ref = 0;
    d.reduce = 1;
    return d;
  };
  auto e1_prod = [&](int R) {
    SmProd d = left ? prod(B_A, R, B_E) : prod(R, B_A, B_E);
    d.reduce = 2;
    return d;
  };
  auto add = [&](int ph, const SmProd& d) { g.prod[ph][g.nprod[ph]++] = d; };
  switch (method) {
    case QPINV_NS: {
      // T = 2I - (side product) and R = I - (side product); X+ = T X
      SmProd d = side_prod(sq(0), -1.0, 2.0);
      d.nout = 2;
      d.out[1] = sq(1);
      d.ca[1] = -1.0;
      d.cg[1] = 1.0;
      add(0, d);
      add(1, update(sq(0)));
      if (e1) {
        add(1, e1_prod(sq(1)));
        g.e1_phase = 1;
      }
      g.nphase = 2;
      break;
    }
    case QPINV_QSAI: {
      // R, S = I + R; R^2; P1 = I + b1 R^2 + R^4, P2 = I + b2 R^2 + R^4; Q = P1 P2; T = S Q; X+ = T X
      SmProd d = side_prod(sq(0), -1.0, 1.0);
      d.nout = 2;
      d.out[1] = sq(1);
      d.ca[1] = -1.0;
      d.cg[1] = 2.0;
      add(0, d);
      add(1, prod(sq(0), sq(0), sq(2)));
      if (e1) {
        add(1, e1_prod(sq(0)));
        g.e1_phase = 1;
      }
      SmProd d4 = prod(sq(2), sq(2), sq(3));
      d4.nout = 2;
      d4.out[1] = sq(4);
      d4.ca[1] = 1.0;
      d4.nin = 1;
      d4.in[0] = sq(2);
      d4.cb[0][0] = kBeta1;
      d4.cb[1][0] = kBeta2;
      d4.cg[0] = d4.cg[1] = 1.0;
      add(2, d4);
      add(3, prod(sq(3), sq(4), sq(5)));
      add(4, prod(sq(1), sq(5), sq(2)));
      add(5, update(sq(2)));
      g.nphase = 6;
      break;
    }
    default: {  // QHPI19
      add(0, side_prod(sq(0), -1.0, 1.0));
      SmProd d2 = prod(sq(0), sq(0), sq(1));  // R^2 and S = R + R^2
      d2.nout = 2;
      d2.out[1] = sq(3);
      d2.ca[1] = 1.0;
      d2.nin = 1;
      d2.in[0] = sq(0);
      d2.cb[1][0] = 1.0;
      add(1, d2);
      if (e1) {
        add(1, e1_prod(sq(0)));
        g.e1_phase = 1;
      }
      SmProd d4 = prod(sq(1), sq(1), sq(2));  // R^4, P1, P2
      d4.nout = 3;
      d4.out[1] = sq(4);
      d4.out[2] = sq(5);
      d4.ca[1] = d4.ca[2] = 1.0;
      d4.nin = 1;
      d4.in[0] = sq(1);
      d4.cb[1][0] = kD1;
      d4.cb[2][0] = kD2;
      d4.cg[1] = d4.cg[2] = 1.0;
      add(2, d4);
      SmProd du = prod(sq(4), sq(5), sq(6));  // U = P1 P2 -> V, W
      du.nout = 2;
      du.out[1] = sq(7);
      du.ca[1] = 1.0;
      du.nin = 2;
      du.in[0] = sq(1);
      du.in[1] = sq(2);
      du.cb[0][0] = kD3;
      du.cb[1][0] = kE1;
      du.cb[1][1] = kE2;
      add(3, du);
      SmProd dg = prod(sq(6), sq(7), sq(4));  // Gamma
      dg.nin = 2;
      dg.in[0] = sq(1);
      dg.in[1] = sq(2);
      dg.cb[0][0] = kC1;
      dg.cb[0][1] = kC2;
      add(4, dg);
      add(5, prod(sq(3), sq(4), sq(5), 1.0, 1.0));  // T = I + S Gamma
      add(6, update(sq(5)));
      g.nphase = 7;
      break;
    }
  }
  return g;
}

// Algorithmic flops of phases [0, last] of one pass: the side product, the update and the E1 product
// (when counted) are s x s x o, the others s^3.
double program_flops(const SmProgram& g, int64_t m, int64_t n, bool left, bool with_e1, int last) {
  const double s = left ? n : m, o = left ? m : n;
  double f = 0.0;
  for (int ph = 0; ph <= last && ph < g.nphase; ++ph)
    for (int q = 0; q < g.nprod[ph]; ++q) {
      const SmProd& d = g.prod[ph][q];
      if (d.reduce == 2 && !with_e1) continue;
      const bool big = d.a == B_A || d.b == B_A || d.reduce != 0;
      f += 32.0 * (big ? s * s * o : s * s * s);
    }
  return f;
}

template <class T>
struct SmMma;
template <>
struct SmMma<double> {
  using type = MM16D;
};
template <>
struct SmMma<float> {
  using type = MM16F;
};

template <class T>
void launch_small(const SmParams<T>* P, int grid, hipStream_t s) {
  hipLaunchKernelGGL((small_solve_kernel<T, typename SmMma<T>::type>), dim3(grid), dim3(SM_THREADS), 0, s, P);
  QP_HIP(hipGetLastError());
}

// Y = X with the element types of the two matrices (same shape).
void sm_convert(const Mat& X, const Mat& Y, hipStream_t s) {
  if (X.dtype == QPINV_F32 && Y.dtype == QPINV_F32)
    convert<float, float>(X.v, Y.v, X.rows, X.cols, s);
  else if (X.dtype == QPINV_F32)
    convert<float, double>(X.v, Y.v, X.rows, X.cols, s);
  else if (Y.dtype == QPINV_F32)
    convert<double, float>(X.v, Y.v, X.rows, X.cols, s);
  else
    convert<double, double>(X.v, Y.v, X.rows, X.cols, s);
}

Mat mat_of(const SmView& v, int dtype) {
  Mat M;
  M.v.p = v.p;
  M.v.rows = v.rows;
  M.v.cols = v.cols;
  M.v.ld = v.ld;
  M.v.ps = v.ps;
  M.rows = v.rows;
  M.cols = v.cols;
  M.dtype = dtype;
  return M;
}

template <class T>
int small_solve_t(Ctx& c, int method, const Mat& A0, int scaling, double am, double tol, int max_iter, int stop,
                  int dtype, const Mat& Xout, qpinv_info& inf, hipStream_t s) {
  const int64_t m = A0.rows, n = A0.cols;
  int side = c.opt.side;
  if (side == QPINV_SIDE_AUTO) side = (m > n) ? QPINV_SIDE_LEFT : QPINV_SIDE_RIGHT;
  const bool left = side == QPINV_SIDE_LEFT;
  const int64_t sd = left ? n : m;
  const bool e1 = stop == STOP_E1_REL;
  inf.side = side;

  Mat A = A0;
  if (A0.dtype != dtype) {
    A = ws_mat(c, "smA", m, n, dtype);
    sm_convert(A0, A, s);
  }
  SmParams<T> P;
  std::memset(&P, 0, sizeof(P));
  auto view = [](const Mat& M) {
    SmView v;
    v.p = M.v.p;
    v.ld = M.v.ld;
    v.ps = M.v.ps;
    v.rows = (int)M.rows;
    v.cols = (int)M.cols;
    return v;
  };
  P.buf[B_A] = view(A);
  P.buf[1] = view(ws_mat(c, "smX0", n, m, dtype));
  P.buf[2] = view(ws_mat(c, "smX1", n, m, dtype));
  for (int k = 0; k < 8; ++k) P.buf[B_SQ + k] = view(ws_mat(c, "smS" + std::to_string(k), sd, sd, dtype));
  P.buf[B_E] = view(ws_mat(c, "smE", m, n, dtype));
  const bool direct = Xout.dtype == dtype;
  P.xout = static_cast<T*>(Xout.v.p);
  P.ldx = Xout.v.ld;
  P.psx = Xout.v.ps;
  P.xout_direct = direct ? 1 : 0;
  P.prog = build_program(method, left, e1);
  P.m = (int)m;
  P.n = (int)n;
  P.scaling = scaling;
  P.power_steps = c.opt.power_steps;
  P.seed = c.opt.power_seed;
  P.alpha_given = am;
  P.mu = am;
  P.stop = stop;
  P.max_iter = max_iter;
  P.tol = tol;
  P.partial = static_cast<double*>(c.ws.get("smPartial", sizeof(double) * 2 * 2 * 2 * SM_MAXG));
  P.state = static_cast<double*>(c.ws.get("smState", sizeof(double) * (S_COUNT + 2)));
  P.bar = reinterpret_cast<unsigned int*>(P.state + S_COUNT);
  constexpr int kTrace = 256;
  if (c.opt.verbose) {
    P.trace = static_cast<unsigned long long*>(c.ws.get("smTrace", sizeof(unsigned long long) * kTrace));
    P.trace_cap = kTrace;
  }
  // The barrier leaves its arrival count at 0 and its give-up flag clear, so the words need clearing only
  // in fresh memory (a new buffer, or the no-allocation scratch, shared by other calls) or after a timeout.
  if (c.no_alloc || c.small_state != P.state) {
    zero_doubles(P.state, S_COUNT + 2, s);  // the record and the barrier words (3 uint32 in 2 doubles)
    c.small_state = c.no_alloc ? nullptr : P.state;
  }
  // grid: the output blocks of the largest phase
  int grid = 1;
  for (int ph = 0; ph < P.prog.nphase; ++ph) {
    int t = 0;
    for (int q = 0; q < P.prog.nprod[ph]; ++q) {
      const SmProd& d = P.prog.prod[ph][q];
      const SmView a = d.a == B_XC || d.a == B_XN ? P.buf[1] : P.buf[d.a];
      const SmView b = d.b == B_XC || d.b == B_XN ? P.buf[1] : P.buf[d.b];
      t += ((a.rows + 15) / 16) * ((b.cols + 15) / 16);
    }
    grid = std::max(grid, t);
  }
  grid = std::min(grid, SM_MAXG);
  // the parameter block goes to device memory through the context's pinned staging area (the kernel reads
  // it through a pointer: indexing it by phase and buffer does not copy it to private memory)
  static_assert(sizeof(SmParams<T>) <= Ctx::kStageBytes, "staging area");
  auto* Pd = static_cast<SmParams<T>*>(c.ws.get("smParams", sizeof(SmParams<T>)));
  std::memcpy(c.hstage, &P, sizeof(P));
  QP_HIP(hipMemcpyAsync(Pd, c.hstage, sizeof(P), hipMemcpyHostToDevice, s));
  launch_small<T>(Pd, grid, s);
  double st[S_COUNT + 2];
  QP_HIP(hipMemcpyAsync(c.hsc, P.state, sizeof(double) * (S_COUNT + 2), hipMemcpyDeviceToHost, s));
  QP_HIP(hipStreamSynchronize(s));
  std::memcpy(st, c.hsc, sizeof(double) * (S_COUNT + 2));
  if (P.trace) {
    std::vector<unsigned long long> tr(kTrace);
    QP_HIP(hipMemcpy(tr.data(), P.trace, sizeof(unsigned long long) * kTrace, hipMemcpyDeviceToHost));
    fprintf(stderr, "[qpinv] small solve, grid %d: barrier times (us from start):", grid);
    for (int i = 1; i < kTrace && tr[i] > tr[0] && tr[i] - tr[0] < 1000000000ull; ++i)
      fprintf(stderr, " %.1f", (tr[i] - tr[0]) * 0.01);
    fprintf(stderr, "\n");
  }
  unsigned int barw[4];
  std::memcpy(barw, st + S_COUNT, sizeof(barw));
  if (barw[2] != 0u) {
    c.small_state = nullptr;
    throw Error(QPINV_ETIMEOUT, "small solve: a grid barrier wait expired");
  }
  const int status = (int)st[S_STATUS];
  inf.alpha_used = st[S_ALPHA];
  if (scaling == QPINV_ALPHA_POWER) {
    inf.sigma1_sq_est = st[S_S1SQ];
    inf.mu_used = am > 0.0 ? am : 1.0;
  }
  if (status == QPINV_ENONFINITE) return status;
  inf.iters = (int)st[S_ITERS];
  (dtype == QPINV_F64 ? inf.iters_f64 : inf.iters_f32) = inf.iters;
  inf.returned = (int)st[S_RETURNED];
  inf.stop_reason = (int)st[S_REASON];
  inf.final_dx_rel = st[S_DXREL];
  inf.e1_rel = st[S_E1];
  // every update's products; with the E1 rule also the E1 products of X_1 .. X_iters and the last pass's
  // phases up to its check
  inf.gemm_flops = inf.iters * program_flops(P.prog, m, n, left, e1 && inf.iters > 1, 99);
  if (e1 && inf.iters > 0) inf.gemm_flops += program_flops(P.prog, m, n, left, true, P.prog.e1_phase);
  c.flops += inf.gemm_flops;
  if (!direct) {
    const Mat Xr = mat_of(P.buf[1 + (int)st[S_RETBUF]], dtype);
    sm_convert(Xr, Xout, s);
    QP_HIP(hipStreamSynchronize(s));
  }
  return status;
}

}  // namespace

bool small_eligible(const Ctx& c, int method, int scaling, int stop, int precision, int64_t m, int64_t n) {
  if (!c.opt.small_path || c.opt.gemm_timing || c.opt.penrose_finish) return false;
  for (int k = 0; k < 3; ++k)
    if (c.opt.force_cfg[k] >= 0) return false;
  if (precision != QPINV_PREC_F64 && precision != QPINV_PREC_F32) return false;
  if (method != QPINV_NS && method != QPINV_QSAI && method != QPINV_QHPI19) return false;
  if (stop != STOP_DX_ABS && stop != STOP_DX_REL && stop != STOP_E1_REL) return false;
  if (scaling != QPINV_ALPHA_POWER && scaling != QPINV_ALPHA_FROB && scaling != QPINV_ALPHA_GIVEN) return false;
  return m >= 1 && n >= 1 && m <= SM_MAXD && n <= SM_MAXD;
}

int small_solve(Ctx& c, int method, const Mat& A0, int scaling, double am, double tol, int max_iter, int stop,
                int precision, const Mat& Xout, qpinv_info& inf, hipStream_t s) {
  if (precision == QPINV_PREC_F64)
    return small_solve_t<double>(c, method, A0, scaling, am, tol, max_iter, stop, QPINV_F64, Xout, inf, s);
  return small_solve_t<float>(c, method, A0, scaling, am, tol, max_iter, stop, QPINV_F32, Xout, inf, s);
}

}  // namespace qp

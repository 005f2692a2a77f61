// Single solves of small matrices (at most 128 per side) in ONE kernel launch.
//
// A solve of a 64 x 48 matrix is a chain of about thirty 48 x 48 products, each a few microseconds of MFMA
// work: launched one by one, with the stop rule read on the host after every update, launch gaps and
// synchronisations take most of the time.  Here one persistent launch runs the whole solve: workgroup 0
// computes ||A||_F, the finiteness check and the power iteration, the grid forms X_0 = alpha A^H, and then
// every product of every update is a phase whose items are 16 x 16 output blocks (all four planes), dealt to
// the workgroups, which meet at a bounded grid barrier after each phase.  Within a block the 8 waves split
// the four output planes and two slices of K (each lane's partial sums meet in LDS), so a product of
// K = 64 costs each wave 32 MFMAs instead of the 256 one wave would issue alone.  The per-element epilogue
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

constexpr int SM_MAXPH = 24;  // phases of one update (QRAPID(N) takes 6 + 2N on the left side, 8 + 2N on the right)

// buffers of the solve: A, the two iterates (current / next resolved per update), 8 side-by-side, the E1
// product A R (left) or R A (right), m x n, and 3 of the iterate's shape, n x m (QRAPID's U, V and nested terms)
enum : int { B_A = 0, B_XC = 1, B_XN = 2, B_SQ = 3, B_E = 11, B_XB = 12, B_N = 15 };

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

// the update's products as the host builds them, phase by phase (products of one phase are independent)
struct SmProgram {
  int nphase;        // phases of one update; the last forms X_{j+1}
  int e1_phase;      // phase whose second product is the E1 product (-1: none)
  int nprod[SM_MAXPH];
  SmProd prod[SM_MAXPH][2];
};

// One product of the program with its buffers resolved.  The iterate buffers swap roles every update and the
// input matrix comes per call, so an operand or epilogue slot that names one of them is left for the kernel
// to bind: `sub` holds 2 bits per slot (A, B, out 0..2, in 0..2 from the low bits up): 0 bound here, 1 the
// current iterate, 2 the next iterate, 3 the input matrix (its strides come per call too).  Both iterate
// buffers have the same strides, which the table holds.
template <class T>
struct SmItem {
  GemmParams<T> g;
  int sub;
};

template <class T>
struct SmParams {
  SmView buf[B_N];       // B_XC / B_XN hold iterate buffers 0 / 1; B_A's pointer and strides come per call
  int nphase, e1_phase;  // the program's shape (as SmProgram) and each product's reduction kind (SmProd)
  int nprod[SM_MAXPH];
  int kind[SM_MAXPH][2];
  int m, n;
  int scaling, power_steps;
  unsigned long long seed;
  double alpha_given, mu;
  int stop, max_iter;
  double tol;
  double* partial;       // [2][2][SM_MAXG * 2]: per item reduction terms (slot by phase kind)
  double* state;         // the set-up's results, broadcast to the workgroups (record slots)
  unsigned int* bar;     // [0] arrivals, [1] Gram blocks written (set-up), [2] give-up flag
  unsigned long long* trace;  // optional (option verbose): workgroup 0 stamps wall_clock64() after each barrier
  int trace_cap;
  // gram = 1 (left side, A^H A) or 2 (right side, A A^H): while workgroup 0 runs the set-up, the others form
  // that Gram matrix (gram_item: the input matrix as both operands, conjugate-transposed as sm_block's CT =
  // gram) into the first output of the update's side product, which for X_0 = alpha A^H is alpha times it;
  // the first update then takes that product's epilogue from it and starts at its second phase.  0: off.
  int gram;
  SmItem<T> gram_item;
  // every product of the program, per phase and product (built on the host, read from LDS by each phase with
  // independent loads).  Last: the host uploads, and the kernel copies, only the program's phases of it.
  SmItem<T> gp[SM_MAXPH][2];
};
// the no-allocation reservation counts 20 KB for the block (noalloc.hip)
static_assert(sizeof(SmParams<double>) <= 20 * 1024 && sizeof(SmParams<float>) <= 20 * 1024, "parameter block size");

// What changes from one call to the next, passed by value: the input matrix, the caller's X (n x m, written
// directly when xout_direct) and the result record in pinned host memory (S_COUNT doubles, written by
// workgroup 0).  The parameter block itself stays in device memory while its bytes do not change.
template <class T>
struct SmCall {
  const T* a;
  int64_t lda, psa;
  T* xout;
  int64_t ldx, psx;
  int xout_direct;
  double* hres;
  unsigned int bar_base;  // the barrier's arrival count when the solve starts
  int pwords;             // 16-byte words of the parameter block in use (up to the program's last phase)
};

// result record, doubles (S_GIVEUP: the barrier's give-up flag as workgroup 0 saw it at the end; S_BARS: the
// grid barriers of the solve, which advance the arrival counter by S_BARS x grid)
enum : int {
  S_STATUS = 0, S_ITERS, S_RETURNED, S_REASON, S_ALPHA, S_S1SQ, S_NORMA2, S_DXREL, S_E1, S_RETBUF, S_NONFINITE,
  S_GIVEUP, S_BARS, S_COUNT
};

constexpr int SM_SU = 8;  // loads in flight per thread in the element-wise passes

// smallest lg with 2^lg >= x (x >= 1)
__device__ __forceinline__ int lg_ceil(int x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }
// plane of row `row` in a plane-major stack of four m-row planes
__device__ __forceinline__ int plane_of(int row, int m) { return (row >= m) + (row >= 2 * m) + (row >= 3 * m); }

// A double moved between lanes of a row of 16 by a DPP control (both halves): no LDS round trip.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_XOR1 = 0xb1;         // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4e;         // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141; // lane i of each 8 <- lane 7 - i
constexpr int DPP_MIRROR = 0x140;      // lane i of each 16 <- lane 15 - i

// Sum over aligned groups of L contiguous lanes (L a power of two <= 64), every lane of a group getting
// the group's sum.  Each step adds two partial sums of equal size (the pairs commute, so every lane of a
// group holds the same bits): quads by DPP, then the quads and halves of a row by mirrors, then the rows by
// shuffles.
__device__ __forceinline__ double group_sum(double x, int L) {
  if (L >= 2) x += dpp_move<DPP_XOR1>(x);
  if (L >= 4) x += dpp_move<DPP_XOR2>(x);
  if (L >= 8) x += dpp_move<DPP_HALF_MIRROR>(x);
  if (L >= 16) x += dpp_move<DPP_MIRROR>(x);
  if (L >= 32) x += __shfl_xor(x, 16, 64);
  if (L >= 64) x += __shfl_xor(x, 32, 64);
  return x;
}

// Sum over the wave, the same bits in every lane: row sums by DPP, then the four rows' sums in a fixed order.
__device__ __forceinline__ double wave_sum(double x) {
  x = group_sum(x, 16);
  const long long b = __double_as_longlong(x);
  double r[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 16 * q);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * q);
    r[q] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  return (r[0] + r[1]) + (r[2] + r[3]);
}

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

// Grid barrier on one arrival counter that only grows during a solve (device memory): barrier k of the
// solve is complete when the counter reaches base + k nblocks (unsigned differences, so it may wrap), so
// the last to arrive has nothing more to do than its own arrival.  Every arrival releases the workgroup's
// writes; the read-modify-writes on the counter form a release sequence, so one acquire after the count is
// reached (by the last arrival's own add or by a relaxed poll) sees every workgroup's writes.  False once
// any workgroup has abandoned a wait (bar[2], the give-up flag, read by every poll: a workgroup whose wait
// needs no poll learns of a give-up at its next wait, and workgroup 0 reports the flag in the record).
__device__ bool sm_sync(unsigned int* bar, unsigned int nblocks, unsigned int base, unsigned int& k) {
  __shared__ int s_ok;
  __syncthreads();
  ++k;
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned int target = k * nblocks;
    const unsigned int arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1u - base;
    if (arrived < target) {
      long long spins = 0;
      while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - base < target) {
        if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > SM_SPIN_MAX) {
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

// workgroup sum of a double, fixed order (every thread gets it)
__device__ __forceinline__ double sm_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  return t;
}

// A buffer of the program for the host: the iterate buffers by their first copy (both have its shape and
// strides), every other buffer as it is.
template <class T>
SmView view_of(const SmParams<T>* P, int b) {
  return P->buf[b == B_XC || b == B_XN ? 1 : b];
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

// The product d of the program with its buffers resolved (host); the slots left for the kernel to bind are
// coded in `sub` and hold no pointer.
template <class T>
SmItem<T> resolve_product(const SmParams<T>* P, const SmProd& d) {
  SmItem<T> it{};
  GemmParams<T>& G = it.g;
  auto code = [](int b) { return b == B_XC ? 1 : b == B_XN ? 2 : b == B_A ? 3 : 0; };
  const SmView a = view_of(P, d.a), b = view_of(P, d.b);
  G.A = code(d.a) ? nullptr : static_cast<const T*>(a.p);
  G.lda = d.a == B_A ? 0 : a.ld;
  G.psa = d.a == B_A ? 0 : a.ps;
  G.B = code(d.b) ? nullptr : static_cast<const T*>(b.p);
  G.ldb = d.b == B_A ? 0 : b.ld;
  G.psb = d.b == B_A ? 0 : b.ps;
  G.M = a.rows;
  G.N = b.cols;
  G.K = a.cols;
  G.tiles_m = (G.M + 15) / 16;
  G.tiles_n = (G.N + 15) / 16;
  G.nout = d.nout;
  G.nin = d.nin;
  G.ref = d.ref;
  it.sub = code(d.a) | code(d.b) << 2;
  for (int t = 0; t < 3; ++t) {
    if (t < d.nout) {
      const SmView o = view_of(P, d.out[t]);
      G.out[t] = code(d.out[t]) ? nullptr : static_cast<T*>(o.p);
      G.ldo[t] = o.ld;
      G.pso[t] = o.ps;
      it.sub |= code(d.out[t]) << (4 + 2 * t);
    }
    if (t < d.nin) {
      const SmView in = view_of(P, d.in[t]);
      G.in[t] = code(d.in[t]) ? nullptr : static_cast<const T*>(in.p);
      G.ldi[t] = in.ld;
      G.psi[t] = in.ps;
      it.sub |= code(d.in[t]) << (10 + 2 * t);
    }
    G.ca[t] = (T)d.ca[t];
    G.cg[t] = (T)d.cg[t];
    for (int u = 0; u < 3; ++u) G.cb[t][u] = (T)d.cb[t][u];
  }
  G.reduce = d.reduce != 0;
  return it;
}

// The slots of a product that the host left unbound (SmItem::sub), bound to this update's iterates xc (current)
// and xn (next) and to the call's input matrix.
template <class T>
__device__ __forceinline__ void sm_bind(GemmParams<T>& G, int sub, T* xc, T* xn, const SmCall<T>& call) {
  auto pick = [&](int code, T* p) { return code == 1 ? xc : code == 2 ? xn : p; };
  const int ca = sub & 3, cb = (sub >> 2) & 3;
  if (ca == 3) {
    G.A = call.a;
    G.lda = call.lda;
    G.psa = call.psa;
  } else if (ca) {
    G.A = pick(ca, nullptr);
  }
  if (cb == 3) {
    G.B = call.a;
    G.ldb = call.lda;
    G.psb = call.psa;
  } else if (cb) {
    G.B = pick(cb, nullptr);
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    G.out[t] = pick((sub >> (4 + 2 * t)) & 3, G.out[t]);
    G.in[t] = pick((sub >> (10 + 2 * t)) & 3, const_cast<T*>(G.in[t]));
  }
}

// One 16 x 16 output block (all four planes) of C = A B with the epilogue.  The block's operands are staged
// in LDS SM_KB deep in k, every thread loading eight elements of each (one memory latency per round): A as
// [plane][row][k], B as [plane][k][column], both padded by one element; the k slots beyond the operands hold
// zeros.  Wave w then takes output plane w % 4 and the k chunks (of 4) with index = w / 4 modulo SM_KSPLIT;
// the slices' partial sums meet in LDS (`red`, which reuses the staging area), and the first slice's waves
// run the epilogue.  The reduction terms are added to s_d, s_x.
constexpr int SM_KB = 64;  // k staged per round (products of K <= 64 take one round)
template <class T>
constexpr int sm_stage_elems() {
  return 4 * 16 * (SM_KB + 1) + 4 * SM_KB * 17;
}

// CT: 0 the operands as given; 1 the left operand is the conjugate transpose of the matrix G.A points at
// (element (r, k) = conj(G.A(k, r)), G.M and G.K the transpose's shape); 2 the same for the right operand.
template <class T, class MM, int CT = 0>
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
    for (int r = 0; r < 4; ++r) epilogue_inputs_overlap(G, p, rb + MM::crow(lane, r), cb + MM::ccol(lane), inv[r]);
  }
  constexpr int NU = 4 * 16 * SM_KB / SM_THREADS;  // staged elements of each operand per thread
  static_assert(NU * SM_THREADS == 4 * 16 * SM_KB && SM_KB == 64, "staging map: 4 planes x 16 x 64 slots");
  for (int k0 = 0; k0 < G.K; k0 += SM_KB) {
    const int kr = G.K - k0 < SM_KB ? G.K - k0 : SM_KB;  // k of this round
    const int kr4 = (kr + 3) & ~3;
    // every load is issued before the first LDS store (one memory latency per round); addresses are clamped
    // into the operands and the values outside them (k beyond the round included) replaced by zeros.  Slot
    // e of A is (plane e / 1024, row (e / 64) % 16, k e % 64), k fastest (rows of A are contiguous in k);
    // slot e of B is (plane e / 1024, k (e / 16) % 64, column e % 16), columns fastest.
    T va[NU], vb[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + u * SM_THREADS;
      const int qa = e >> 10, ra = (e >> 6) & 15, kka = e & 63;
      const int row = rb + ra;
      const bool oka = kka < kr && row < G.M;
      const int qb = e >> 10, kkb = (e >> 4) & 63, cc = e & 15;
      const int col = cb + cc;
      const bool okb = kkb < kr && col < G.N;
      const int64_t offa = CT == 1 ? (int64_t)(k0 + kka) * G.lda + row : (int64_t)row * G.lda + (k0 + kka);
      const int64_t offb = CT == 2 ? (int64_t)col * G.ldb + (k0 + kkb) : (int64_t)(k0 + kkb) * G.ldb + col;
      va[u] = gload(G.A, oka ? qa * G.psa + offa : 0);
      vb[u] = gload(G.B, okb ? qb * G.psb + offb : 0);
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + u * SM_THREADS;
      const bool oka = (e & 63) < kr && rb + ((e >> 6) & 15) < G.M;
      const bool okb = ((e >> 4) & 63) < kr && cb + (e & 15) < G.N;
      // a conjugated operand's planes i, j, k change sign
      const T xa = CT == 1 && (e >> 10) > 0 ? -va[u] : va[u];
      const T xb = CT == 2 && (e >> 10) > 0 ? -vb[u] : vb[u];
      As[((e >> 10) * 16 + ((e >> 6) & 15)) * (SM_KB + 1) + (e & 63)] = oka ? xa : T(0);
      Bs[((e >> 10) * SM_KB + ((e >> 4) & 63)) * 17 + (e & 15)] = okb ? xb : T(0);
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

// w = c A v (ADJ = false; v: 4 n, w: 4 m) or w = c A^H v (ADJ = true; v: 4 m, w: 4 n), planes [p][i], v
// and w in LDS, A in LDS or in device memory (the address space of AP).  Element i of w is the sum of a group
// of L lanes (L a power of two, the largest with one group per row; groups are contiguous within a wave),
// lane l of the group taking the columns l, l + L, ...; the group's sums meet in a fixed order (group_sum).
// Returns the sum of |w_i|^2 over the rows this lane wrote (nonzero on the groups' first lanes only).
template <bool ADJ, class AP>
__device__ __forceinline__ double sm_gemv(AP a, int64_t lda, int64_t psa, int m, int n, double c, const double* v,
                                          double* w, double* dot = nullptr) {
  const int tid = threadIdx.x;
  const int rows = ADJ ? n : m, cols = ADJ ? m : n;
  const int lgl = min(6, 31 - __clz((int)blockDim.x / rows));  // rows <= 128, 512 threads: L >= 4
  const int L = 1 << lgl, i = tid >> lgl, l = tid & (L - 1);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < rows) {
#pragma unroll 2
    for (int j = l; j < cols; j += L) {
      // element (i, j) of A or of A^H (= conj of A's (j, i))
      const int64_t off = ADJ ? (int64_t)j * lda + i : (int64_t)i * lda + j;
      double aq[4], vq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        aq[q] = (double)a[q * psa + off];
        vq[q] = v[q * cols + j];
      }
      if (ADJ) {
        aq[1] = -aq[1];
        aq[2] = -aq[2];
        aq[3] = -aq[3];
      }
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
#pragma unroll
        for (int q = 0; q < 4; ++q) s[pl] += qsign(pl, q) * aq[q] * vq[pl ^ q];
    }
  }
#pragma unroll
  for (int pl = 0; pl < 4; ++pl) s[pl] = group_sum(s[pl], L);
  double nrm = 0.0, vw = 0.0;
  if (i < rows && l == 0) {
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      const double x = c * s[pl];
      w[pl * rows + i] = x;
      nrm += x * x;
      if (dot) vw += v[pl * cols + i] * x;
    }
  }
  if (dot) *dot = vw;
  return nrm;
}

// Sum over the workgroup of one double per thread, through per-wave partials in sh[0 .. waves): the waves'
// sums are written, then after the barrier every thread adds them in wave order.
__device__ __forceinline__ double sm_sum_partials(const double* sh) {
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  return t;
}

// Sum of count <= 64 per-tile values v[t * stride], one load per lane and a fixed-order wave sum: every
// workgroup adds the same pairs in the same order, so all of them get the same bits.
static_assert((SM_MAXD / 16) * (SM_MAXD / 16) <= 64, "a product's output blocks fit one wave");
__device__ __forceinline__ double sm_tile_sum(const double* v, int count, int stride) {
  const int lane = threadIdx.x & 63;
  const double x = gload(v, (int64_t)(lane < count ? lane : 0) * stride);
  return wave_sum(lane < count ? x : 0.0);
}

// The power iteration of the classical scaling, run by one workgroup: v_0 from the seeded generator, then
// per step v <- v / ||v||, w = A v, sigma_1^2 estimate ||w||^2, v <- A^H w.  The normalisation is folded into
// the product (w = (A v) / ||v||), ||v||^2 and ||w||^2 ride along as wave partials, so a step is two
// workgroup barriers.  Returns the last step's ||w||^2.
template <class AP>
__device__ __forceinline__ double sm_power(AP a, int64_t lda, int64_t psa, int m, int n, int steps, uint64_t seed, double* vs,
                           double* wsv, double* shv, double* shw) {
  const int tid = threadIdx.x, wv = tid >> 6;
  double vv = 0.0;
  for (int e = tid; e < 4 * n; e += blockDim.x) {
    const double x = (double)(sm_splitmix64((uint64_t)e, seed) >> 11) * 0x1p-52 - 1.0;
    vs[e] = x;
    vv += x * x;
  }
  vv = wave_sum(vv);
  if ((tid & 63) == 0) shv[wv] = vv;
  __syncthreads();
  double s1sq = 0.0;
  for (int it = 0; it < steps; ++it) {
    const double inv = 1.0 / sqrt(sm_sum_partials(shv));
    const double ww = wave_sum(sm_gemv<false>(a, lda, psa, m, n, inv, vs, wsv));
    if ((tid & 63) == 0) shw[wv] = ww;
    __syncthreads();
    s1sq = sm_sum_partials(shw);
    const double nv = wave_sum(sm_gemv<true>(a, lda, psa, m, n, 1.0, wsv, vs));
    if ((tid & 63) == 0) shv[wv] = nv;
    __syncthreads();
  }
  return s1sq;
}

// The same power iteration on the Gram matrix Gm = A^H A (n x n): per step v <- v / ||v||, u = Gm v, the
// sigma_1^2 estimate (v . u) / ||v|| (= ||A v||^2 / ||v||^2 in exact arithmetic), v <- u, so one product and one
// workgroup barrier per step.  The per-wave partials alternate between two slots of shv / shd (8 waves each),
// so a wave that starts the next step cannot overwrite what a slower one still reads.
static_assert(SM_THREADS / 64 == 8, "two slots of 8 per-wave partials in sh[32]");
template <class AP>
__device__ __forceinline__ double sm_power_gram(AP g, int64_t ldg, int64_t psg, int n, int steps, uint64_t seed, double* vs,
                                double* us, double* shv, double* shd) {
  const int tid = threadIdx.x, wv = tid >> 6;
  double vv = 0.0;
  for (int e = tid; e < 4 * n; e += blockDim.x) {
    const double x = (double)(sm_splitmix64((uint64_t)e, seed) >> 11) * 0x1p-52 - 1.0;
    vs[e] = x;
    vv += x * x;
  }
  vv = wave_sum(vv);
  if ((tid & 63) == 0) shv[wv] = vv;
  __syncthreads();
  double s1sq = 0.0;
  double *v = vs, *u = us;
  for (int it = 0; it < steps; ++it) {
    const int rd = (it & 1) * 8, wr = 8 - rd;
    const double inv = 1.0 / sqrt(sm_sum_partials(shv + rd));
    double dot = 0.0;
    const double nu = wave_sum(sm_gemv<false>(g, ldg, psg, n, n, inv, v, u, &dot));
    dot = wave_sum(dot);
    if ((tid & 63) == 0) {
      shv[wr + wv] = nu;
      shd[rd + wv] = dot;
    }
    __syncthreads();
    s1sq = sm_sum_partials(shd + rd) * inv;
    double* t = v;
    v = u;
    u = t;
  }
  return s1sq;
}

// Waits (thread 0, bounded by the give-up rule of sm_sync) until *cnt >= target, then acquires.  False if the
// wait gave up (the flag is raised; the next grid barrier then returns false everywhere).
__device__ bool sm_wait_count(unsigned int* cnt, unsigned int target, unsigned int* bar) {
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    int ok = 1;
    long long spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > SM_SPIN_MAX) {
        __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// The result record, written into pinned host memory by one thread at the end of the solve.
template <class T>
__device__ void sm_record(const SmParams<T>* P, double* hres, int status, int iters, int returned, int reason, double alpha,
                          double s1sq, double fro, double dx_rel, double e1_rel, int ret_buf, double bad,
                          unsigned int bars) {
  double r[S_COUNT];
  r[S_STATUS] = status;
  r[S_ITERS] = iters;
  r[S_RETURNED] = returned;
  r[S_REASON] = reason;
  r[S_ALPHA] = alpha;
  r[S_S1SQ] = s1sq;
  r[S_NORMA2] = fro;
  r[S_DXREL] = dx_rel;
  r[S_E1] = e1_rel;
  r[S_RETBUF] = ret_buf;
  r[S_NONFINITE] = bad;
  r[S_GIVEUP] = __hip_atomic_load(&P->bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  r[S_BARS] = bars;
#pragma unroll
  for (int k = 0; k < S_COUNT; ++k) gstore(hres, k, r[k]);
}

template <class T, class MM>
__global__ void __launch_bounds__(SM_THREADS) small_solve_kernel(const SmParams<T>* __restrict__ Pg, const SmCall<T> call) {
  // one LDS area: the operand staging of a product (one K round), the K-slice exchange after it ((SM_KSPLIT - 1)
  // x 4 planes x 64 lanes of accumulators), and in the set-up a copy of A when A fits
  constexpr int RED_BYTES = (SM_KSPLIT - 1) * 4 * 64 * (int)sizeof(typename MM::Acc);
  constexpr int STAGE_BYTES = sm_stage_elems<T>() * (int)sizeof(T);
  constexpr int SETUP_BYTES = 120 * 1024;  // a copy of A of up to 120 KB
  constexpr int LDS_BYTES0 = STAGE_BYTES > RED_BYTES ? STAGE_BYTES : RED_BYTES;
  constexpr int LDS_BYTES = LDS_BYTES0 > SETUP_BYTES ? LDS_BYTES0 : SETUP_BYTES;
  __shared__ __attribute__((aligned(16))) unsigned char lds[LDS_BYTES];
  typename MM::Acc* const red = reinterpret_cast<typename MM::Acc*>(lds);
  T* const stage = reinterpret_cast<T*>(lds);
  T* const acopy = reinterpret_cast<T*>(lds);
  constexpr int ACOPY_ELEMS = LDS_BYTES / (int)sizeof(T);
  __shared__ double sh[32];
  __shared__ double vs[4 * SM_MAXD], wsv[4 * SM_MAXD];
  // the parameter block up to the program's last phase (call.pwords 16-byte words), read once from device
  // memory (phases index it by product); every thread issues its loads before its first LDS store, one round
  // trip for the whole block
  constexpr int PV = (int)((sizeof(SmParams<T>) + 15) / 16), PU = (PV + SM_THREADS - 1) / SM_THREADS;
  __shared__ uint4 pcopy[PV];
  {
    const uint4* src = reinterpret_cast<const uint4*>(Pg);
    const int pw = call.pwords < PV ? call.pwords : PV;
    uint4 v[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int i = (int)threadIdx.x + u * SM_THREADS;
      v[u] = src[i < pw ? i : 0];
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int i = (int)threadIdx.x + u * SM_THREADS;
      if (i < pw) pcopy[i] = v[u];
    }
    __syncthreads();
  }
  const SmParams<T>* const P = reinterpret_cast<const SmParams<T>*>(pcopy);
  const int tid = threadIdx.x;
  const unsigned int G = gridDim.x;
  unsigned int nbar = 0;  // grid barriers passed in this solve
  int nstamp = 0;
  auto stamp = [&]() {
    if (P->trace && blockIdx.x == 0 && tid == 0 && nstamp < P->trace_cap) P->trace[nstamp] = wall_clock64();
    ++nstamp;
  };
  stamp();
  const int m = P->m, n = P->n;
  SmView A = P->buf[B_A];
  A.p = const_cast<T*>(call.a);
  A.ld = call.lda;
  A.ps = call.psa;
  const T* a = static_cast<const T*>(A.p);

  // ---------------------------------------------------------------- set-up (workgroup 0)
  if (blockIdx.x == 0) {
    // one pass over A: ||A||_F^2, the non-finite count and, for the power iteration, a copy of A in LDS
    // when it fits (every power step reads all of it twice).  Rows (plane-major, 4 m of them) are mapped
    // on slots of 2^lgw >= n columns, so a slot's row and column are a shift and a mask, and every thread
    // has SM_SU loads in flight at a time.
    // the LDS copy's row stride is n rounded up to 8 mod 16 elements when that fits: the lanes of a wave that
    // read one column in different rows (both products of a power step) then fall on different banks
    const int ldp = ((n + 7) >> 4) * 16 + 8, ldc = 4 * m * ldp <= ACOPY_ELEMS ? ldp : n;
    // with the Gram matrix A^H A formed meanwhile (left side), the power steps run on it instead (padded the
    // same way in LDS), one product per step
    const bool gram_pw = P->scaling == QPINV_ALPHA_POWER && P->gram == 1 && 4 * n * ldp <= ACOPY_ELEMS;
    const bool in_lds = P->scaling == QPINV_ALPHA_POWER && !gram_pw && 4 * m * ldc <= ACOPY_ELEMS;
    double fro = 0.0, bad = 0.0;
    {
      const int lgw = lg_ceil(n), slots = (4 * m) << lgw;
      for (int e0 = tid; e0 < slots; e0 += SM_SU * (int)blockDim.x) {
        T v[SM_SU];
#pragma unroll
        for (int u = 0; u < SM_SU; ++u) {
          const int e = e0 + u * (int)blockDim.x, row = e >> lgw, c = e & ((1 << lgw) - 1);
          const int pl = plane_of(row, m);
          const bool ok = e < slots && c < n;
          v[u] = gload(a, ok ? pl * A.ps + (int64_t)(row - pl * m) * A.ld + c : 0);
        }
#pragma unroll
        for (int u = 0; u < SM_SU; ++u) {
          const int e = e0 + u * (int)blockDim.x, row = e >> lgw, c = e & ((1 << lgw) - 1);
          if (e < slots && c < n) {
            const double x = (double)v[u];
            if (!__builtin_isfinite(x)) bad += 1.0;
            fro += x * x;
            if (in_lds) acopy[row * ldc + c] = v[u];
          }
        }
      }
    }
    fro = sm_sum(fro, sh);
    bad = sm_sum(bad, sh);
    double alpha = 0.0, s1sq = 0.0;
    if (bad == 0.0 && fro > 0.0) {
      if (gram_pw) {
        const GemmParams<T>& gg = P->gram_item.g;
        if (sm_wait_count(&P->bar[1], (unsigned int)(gg.tiles_m * gg.tiles_n), P->bar)) {
          // Gm into LDS: its 4 n rows on slots of 2^lgw >= n columns, SM_SU loads in flight per thread
          const T* gp = gg.out[0];
          const int lgw = lg_ceil(n), slots = (4 * n) << lgw;
          for (int e0 = tid; e0 < slots; e0 += SM_SU * (int)blockDim.x) {
            T v[SM_SU];
#pragma unroll
            for (int u = 0; u < SM_SU; ++u) {
              const int e = e0 + u * (int)blockDim.x, row = e >> lgw, c = e & ((1 << lgw) - 1), pl = plane_of(row, n);
              v[u] = gload(gp, e < slots && c < n ? pl * gg.pso[0] + (int64_t)(row - pl * n) * gg.ldo[0] + c : 0);
            }
#pragma unroll
            for (int u = 0; u < SM_SU; ++u) {
              const int e = e0 + u * (int)blockDim.x, row = e >> lgw, c = e & ((1 << lgw) - 1);
              if (e < slots && c < n) acopy[row * ldp + c] = v[u];
            }
          }
          __syncthreads();
          s1sq = sm_power_gram((const __attribute__((address_space(3))) T*)acopy, ldp, (int64_t)n * ldp, n,
                               P->power_steps, P->seed, vs, wsv, sh, sh + 16);
          alpha = (P->mu > 0.0 ? P->mu : 1.0) / s1sq;
        }
      } else if (P->scaling == QPINV_ALPHA_POWER) {
        if (in_lds)
          s1sq = sm_power((const __attribute__((address_space(3))) T*)acopy, ldc, (int64_t)m * ldc, m, n,
                          P->power_steps, P->seed, vs, wsv, sh, sh + 16);
        else
          s1sq = sm_power((const __attribute__((address_space(1))) T*)a, A.ld, A.ps, m, n,
                          P->power_steps, P->seed, vs, wsv, sh, sh + 16);
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
  } else if (P->gram != 0) {
    // the Gram matrix meanwhile, by workgroups 1 .. (its blocks read only A)
    GemmParams<T> gq = P->gram_item.g;
    sm_bind(gq, P->gram_item.sub, static_cast<T*>(P->buf[1].p), static_cast<T*>(P->buf[2].p), call);
    make_uniform(gq);
    unsigned int done_blocks = 0;
    for (int t = blockIdx.x - 1; t < gq.tiles_m * gq.tiles_n; t += G - 1) {
      double s_d = 0.0, s_x = 0.0;
      if (P->gram == 1)
        sm_block<T, MM, 1>(gq, t / gq.tiles_n, t % gq.tiles_n, stage, red, s_d, s_x);
      else
        sm_block<T, MM, 2>(gq, t / gq.tiles_n, t % gq.tiles_n, stage, red, s_d, s_x);
      ++done_blocks;
    }
    // the blocks are counted (released) for workgroup 0, which may run the power steps on them
    if (tid == 0 && done_blocks)
      __hip_atomic_fetch_add(&P->bar[1], done_blocks, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!sm_sync(P->bar, G, call.bar_base, nbar)) return;
  stamp();
  // every Gram block was counted before the barrier: the count starts from zero in the next solve
  if (P->gram != 0 && blockIdx.x == 0 && tid == 0) __hip_atomic_store(&P->bar[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double bad = __hip_atomic_load(&P->state[S_NONFINITE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double fro = __hip_atomic_load(&P->state[S_NORMA2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double alpha = __hip_atomic_load(&P->state[S_ALPHA], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (bad != 0.0) {
    if (blockIdx.x == 0 && tid == 0)
      sm_record(P, call.hres, QPINV_ENONFINITE, 0, 0, QPINV_REASON_TOL, alpha, P->state[S_S1SQ], fro, 0.0, -1.0, 0, bad,
                nbar);
    return;
  }
  const double normA = sqrt(fro);
  const int gtid = blockIdx.x * blockDim.x + tid, gthreads = G * blockDim.x;

  // ---------------------------------------------------------------- X_0 = alpha A^H into iterate 0
  {
    // X_0 element (r, c) = alpha conj(A(c, r)); X_0's 4 n rows on slots of 2^lgw >= m columns
    const SmView X0 = P->buf[1];
    T* x = static_cast<T*>(X0.p);
    const int lgw = lg_ceil(m), slots = (4 * n) << lgw;
    for (int e0 = gtid; e0 < slots; e0 += SM_SU * gthreads) {
      T v[SM_SU];
#pragma unroll
      for (int u = 0; u < SM_SU; ++u) {
        const int e = e0 + u * gthreads, row = e >> lgw, c = e & ((1 << lgw) - 1), pl = plane_of(row, n);
        v[u] = gload(a, e < slots && c < m ? pl * A.ps + (int64_t)c * A.ld + (row - pl * n) : 0);
      }
#pragma unroll
      for (int u = 0; u < SM_SU; ++u) {
        const int e = e0 + u * gthreads, row = e >> lgw, c = e & ((1 << lgw) - 1), pl = plane_of(row, n);
        if (e < slots && c < m)
          gstore(x, pl * X0.ps + (int64_t)(row - pl * n) * X0.ld + c, (T)(alpha * (double)(pl == 0 ? v[u] : -v[u])));
      }
    }
  }
  if (P->gram != 0 && normA > 0.0) {
    // the first update's side product X_0 A (A X_0) = alpha times the Gram matrix: its epilogue applied to
    // alpha G element by element (in place over G, which is its first output), the values loaded first
    GemmParams<T> g0 = P->gp[0][0].g;
    sm_bind(g0, P->gp[0][0].sub, static_cast<T*>(P->buf[1].p), static_cast<T*>(P->buf[2].p), call);
    make_uniform(g0);
    constexpr int EPT = 4 * 16 * 16 / SM_THREADS;
    static_assert(EPT * SM_THREADS == 4 * 16 * 16, "a 16 x 16 block of four planes per pass");
    for (int t = blockIdx.x; t < g0.tiles_m * g0.tiles_n; t += G) {
      const int rb = (t / g0.tiles_n) * 16, cb = (t % g0.tiles_n) * 16;
      T gv[EPT];
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int e = tid + u * SM_THREADS, p = e >> 8, row = rb + ((e >> 4) & 15), col = cb + (e & 15);
        const bool ok = row < g0.M && col < g0.N;
        gv[u] = gload(g0.out[0], ok ? p * g0.pso[0] + (int64_t)row * g0.ldo[0] + col : 0);
      }
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int e = tid + u * SM_THREADS, p = e >> 8, row = rb + ((e >> 4) & 15), col = cb + (e & 15);
        const T inv[3] = {T(0), T(0), T(0)};
        double s_d = 0.0, s_x = 0.0;
        epilogue_apply(g0, p, row, col, (T)(alpha * (double)gv[u]), inv, s_d, s_x);
      }
    }
  }
  if (!sm_sync(P->bar, G, call.bar_base, nbar)) return;
  stamp();

  // ---------------------------------------------------------------- updates
  StopController ctl(P->stop, P->tol);
  const bool e1 = P->stop == STOP_E1_REL;
  int cur = 0, j = 0;
  int status = QPINV_OK, reason = QPINV_REASON_TOL, ret_buf = 0, ret_j = 0;
  double dx_rel = 0.0, e1_rel = -1.0;
  bool done = normA == 0.0;  // A = 0: X_0 = 0 is the pseudoinverse
  while (!done) {
    T* const xc = static_cast<T*>(P->buf[1 + cur].p);
    T* const xn = static_cast<T*>(P->buf[2 - cur].p);
    for (int ph = j == 0 && P->gram != 0 ? 1 : 0; ph < P->nphase && !done; ++ph) {
      const int np = P->nprod[ph];
      // output blocks of the phase's products (X_0's E1 is never needed)
      int tiles[2] = {0, 0};
      for (int q = 0; q < 2; ++q) {
        if (q >= np || (q == 1 && ph == P->e1_phase && j == 0)) continue;
        tiles[q] = P->gp[ph][q].g.tiles_m * P->gp[ph][q].g.tiles_n;
      }
      const int total = tiles[0] + tiles[1];
      for (int item = blockIdx.x; item < total; item += G) {
        const int q = item < tiles[0] ? 0 : 1;
        const int t = item - (q ? tiles[0] : 0);
        GemmParams<T> gq = P->gp[ph][q].g;
        sm_bind(gq, P->gp[ph][q].sub, xc, xn, call);
        make_uniform(gq);
        double s_d = 0.0, s_x = 0.0;
        sm_block<T, MM>(gq, t / gq.tiles_n, t % gq.tiles_n, stage, red, s_d, s_x);
        const int kind = P->kind[ph][q];
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
      if (!sm_sync(P->bar, G, call.bar_base, nbar)) return;
      stamp();
      if (e1 && ph == P->e1_phase && j >= 1) {
        // ||A X_j A - A||_F / ||A||_F from the tiles of the E1 product, summed in tile order
        const double s = sm_tile_sum(P->partial + 2 * 2 * SM_MAXG + 1, tiles[1], 2);
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
      if (done || ph != P->nphase - 1) continue;
      // the update X_{j+1} = X_nxt is formed: its change norms summed over the tiles, then the stop rule
      const int tu = P->kind[ph][0] == 1 ? tiles[0] : 0;
      const double d2 = sm_tile_sum(P->partial, tu, 2), x2 = sm_tile_sum(P->partial + 1, tu, 2);
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
  if (call.xout_direct) {
    const SmView Xr = P->buf[1 + ret_buf];
    const T* x = static_cast<const T*>(Xr.p);
    const int lgw = lg_ceil(m), slots = (4 * n) << lgw;
    for (int e0 = gtid; e0 < slots; e0 += SM_SU * gthreads) {
      T v[SM_SU];
#pragma unroll
      for (int u = 0; u < SM_SU; ++u) {
        const int e = e0 + u * gthreads, row = e >> lgw, c = e & ((1 << lgw) - 1), pl = plane_of(row, n);
        v[u] = gload(x, e < slots && c < m ? pl * Xr.ps + (int64_t)(row - pl * n) * Xr.ld + c : 0);
      }
#pragma unroll
      for (int u = 0; u < SM_SU; ++u) {
        const int e = e0 + u * gthreads, row = e >> lgw, c = e & ((1 << lgw) - 1), pl = plane_of(row, n);
        if (e < slots && c < m) gstore(call.xout, pl * call.psx + (int64_t)(row - pl * n) * call.ldx + c, v[u]);
      }
    }
  }
  if (blockIdx.x == 0 && tid == 0)
    sm_record(P, call.hres, status, j, ret_j, reason, alpha, P->state[S_S1SQ], fro, dx_rel, e1_rel, ret_buf, bad, nbar);
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

int xb(int k) { return B_XB + k; }

// Phases of one QRAPID(N) update (Algorithm 1): 6 + 2N on the left side, 8 + 2N on the right.
int qrapid_phases(int N, bool left) { return (left ? 6 : 8) + 2 * N; }

// Products of one update of `method` on `side` (left: R = I - X A, X+ = T X; right: R = I - A X, X+ = X T).
SmProgram build_program(int method, int order, bool left, bool e1) {
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
    case QPINV_QRAPID: {
      // Algorithm 1 with N = order nested steps.  Left: Q = X A, H1 = 7I - Q, H2 = 15I - Q H1, F = 13I - Q H2,
      // U = F X / 4, V = U + X - Q U, Z = W + Y - (Y A) W (N times), X+ = Z + X - Q Z.  Right: P = A X, the same
      // Horner factors from P, U = X F / 4, V = U + X (I - A U), Z = W + Y (I - A W), X+ = Z + X (I - A Z).
      // R = I - Q (I - P) rides on the first product for the E1 rule.
      const int N = order;
      SmProd d = side_prod(sq(0), 1.0, 0.0);
      d.nout = e1 ? 3 : 2;
      d.out[1] = sq(1);
      d.ca[1] = -1.0;
      d.cg[1] = 7.0;
      if (e1) {
        d.out[2] = sq(4);
        d.ca[2] = -1.0;
        d.cg[2] = 1.0;
      }
      add(0, d);
      add(1, prod(sq(0), sq(1), sq(2), -1.0, 15.0));
      if (e1) {
        add(1, e1_prod(sq(4)));
        g.e1_phase = 1;
      }
      add(2, prod(sq(0), sq(2), sq(1), -1.0, 13.0));  // F into H1
      int ph = 3;
      auto plus = [](SmProd d2, int in0, int in1, double b0, double b1) {
        d2.nin = in1 < 0 ? 1 : 2;
        d2.in[0] = in0;
        d2.cb[0][0] = b0;
        if (in1 >= 0) {
          d2.in[1] = in1;
          d2.cb[0][1] = b1;
        }
        return d2;
      };
      int Y = xb(0), W = xb(1), F = xb(2);
      if (left) {
        add(ph++, prod(sq(1), B_XC, xb(0), 0.25));                                   // U
        add(ph++, plus(prod(sq(0), xb(0), xb(1), -1.0), xb(0), B_XC, 1.0, 1.0));   // V
        for (int l = 0; l < N; ++l) {
          add(ph++, prod(Y, B_A, sq(3)));                                           // Y A
          add(ph++, plus(prod(sq(3), W, F, -1.0), W, Y, 1.0, 1.0));                 // Z
          const int freed = Y;
          Y = W;
          W = F;
          F = freed;
        }
        SmProd u = plus(prod(sq(0), W, B_XN, -1.0), W, B_XC, 1.0, 1.0);
        u.ref = 1;
        u.reduce = 1;
        add(ph++, u);
      } else {
        add(ph++, prod(B_XC, sq(1), xb(0), 0.25));                      // U
        add(ph++, prod(B_A, xb(0), sq(3), -1.0, 1.0));                  // I - A U
        add(ph++, plus(prod(B_XC, sq(3), xb(1)), xb(0), -1, 1.0, 0.0));  // V
        for (int l = 0; l < N; ++l) {
          add(ph++, prod(B_A, W, sq(3), -1.0, 1.0));                    // I - A W
          add(ph++, plus(prod(Y, sq(3), F), W, -1, 1.0, 0.0));          // Z
          const int freed = Y;
          Y = W;
          W = F;
          F = freed;
        }
        add(ph++, prod(B_A, W, sq(3), -1.0, 1.0));  // I - A Z
        SmProd u = plus(prod(B_XC, sq(3), B_XN), W, B_XC, 1.0, 0.0);
        u.ref = 1;
        u.reduce = 1;
        add(ph++, u);
      }
      g.nphase = ph;
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

// Algorithmic flops of phases [0, last] of one pass: 32 M N K per quaternion product, from the buffers'
// shapes (A m x n, the iterates and the B_XB buffers n x m, the side-by-side s x s, the E1 product m x n).
double program_flops(const SmProgram& g, int64_t m, int64_t n, bool left, bool with_e1, int last) {
  const double s = left ? n : m;
  auto rows = [&](int b) { return b == B_A || b == B_E ? (double)m : b < B_SQ || b >= B_XB ? (double)n : s; };
  auto cols = [&](int b) { return b == B_A || b == B_E ? (double)n : b < B_SQ || b >= B_XB ? (double)m : s; };
  double f = 0.0;
  for (int ph = 0; ph <= last && ph < g.nphase; ++ph)
    for (int q = 0; q < g.nprod[ph]; ++q) {
      const SmProd& d = g.prod[ph][q];
      if (d.reduce == 2 && !with_e1) continue;
      f += 32.0 * rows(d.a) * cols(d.b) * cols(d.a);
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
void launch_small(const SmParams<T>* P, const SmCall<T>& call, int grid, hipStream_t s) {
  hipLaunchKernelGGL((small_solve_kernel<T, typename SmMma<T>::type>), dim3(grid), dim3(SM_THREADS), 0, s, P, call);
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
int small_solve_t(Ctx& c, int method, int order, const Mat& A0, int scaling, double am, double tol, int max_iter,
                  int stop, int dtype, const Mat& Xout, qpinv_info& inf, hipStream_t s) {
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
  SmCall<T> call;
  call.a = static_cast<const T*>(A.v.p);
  call.lda = A.v.ld;
  call.psa = A.v.ps;
  P.buf[B_A].p = nullptr;  // per call
  P.buf[B_A].ld = P.buf[B_A].ps = 0;
  P.buf[1] = view(ws_mat(c, "smX0", n, m, dtype));  // one shape, so the same strides (SmItem relies on it)
  P.buf[2] = view(ws_mat(c, "smX1", n, m, dtype));
  for (int k = 0; k < 8; ++k) P.buf[B_SQ + k] = view(ws_mat(c, "smS" + std::to_string(k), sd, sd, dtype));
  P.buf[B_E] = view(ws_mat(c, "smE", m, n, dtype));
  if (method == QPINV_QRAPID)
    for (int k = 0; k < 3; ++k) P.buf[B_XB + k] = view(ws_mat(c, "smB" + std::to_string(k), n, m, dtype));
  const bool direct = Xout.dtype == dtype;
  call.xout = static_cast<T*>(Xout.v.p);
  call.ldx = Xout.v.ld;
  call.psx = Xout.v.ps;
  call.xout_direct = direct ? 1 : 0;
  const SmProgram prog = build_program(method, order, left, e1);
  P.nphase = prog.nphase;
  P.e1_phase = prog.e1_phase;
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
  for (int ph = 0; ph < prog.nphase; ++ph) {
    P.nprod[ph] = prog.nprod[ph];
    for (int q = 0; q < prog.nprod[ph]; ++q) {
      P.kind[ph][q] = prog.prod[ph][q].reduce;
      P.gp[ph][q] = resolve_product(&P, prog.prod[ph][q]);
    }
  }
  constexpr int kTrace = 256;
  if (c.opt.verbose) {
    P.trace = static_cast<unsigned long long*>(c.ws.get("smTrace", sizeof(unsigned long long) * kTrace));
    P.trace_cap = kTrace;
  }
  // The barrier's arrival counter keeps the count the previous solve left (passed as the next one's base)
  // and its give-up flag stays clear, so the words need clearing only in fresh memory (a new buffer, or
  // the no-allocation scratch, shared by other calls) or after a timeout.
  if (c.no_alloc || c.small_state != P.state) {
    zero_doubles(P.state, S_COUNT + 2, s);  // the broadcast slots and the barrier words (3 uint32 in 2 doubles)
    c.small_state = c.no_alloc ? nullptr : P.state;
    c.small_bar_base = 0;
  }
  if (c.opt.fault_small_giveup) {
    // test hook: every workgroup sees the flag at its first barrier and leaves (no wait runs out)
    static const unsigned int kRaised = 1u;
    QP_HIP(hipMemcpyAsync(P.bar + 2, &kRaised, sizeof(kRaised), hipMemcpyHostToDevice, s));
  }
  // grid: the output blocks of the largest phase
  int grid = 1;
  for (int ph = 0; ph < prog.nphase; ++ph) {
    int t = 0;
    for (int q = 0; q < prog.nprod[ph]; ++q) t += P.gp[ph][q].g.tiles_m * P.gp[ph][q].g.tiles_n;
    grid = std::max(grid, t);
  }
  grid = std::min(grid, SM_MAXG);
  // The Gram matrix during the set-up (FP64; a side product of one plain output set, and enough other
  // workgroups for one Gram block each).
  {
    const SmProd& d = prog.prod[0][0];
    const int st = (int)((sd + 15) / 16) * (int)((sd + 15) / 16);
    if (c.opt.small_gram && dtype == QPINV_F64 && prog.nprod[0] == 1 && d.nin == 0 && d.reduce == 0 && grid - 1 >= st) {
      SmProd dg = d;
      dg.a = dg.b = B_A;
      dg.nout = 1;
      dg.ca[0] = 1.0;
      dg.cg[0] = 0.0;
      dg.ref = 3;
      P.gram_item = resolve_product(&P, dg);
      GemmParams<T>& g = P.gram_item.g;
      g.M = g.N = (int)sd;
      g.K = (int)(left ? m : n);
      g.tiles_m = g.tiles_n = (int)((sd + 15) / 16);
      P.gram = left ? 1 : 2;
    }
  }
  // The parameter block goes to device memory through the context's pinned staging area, and only when
  // its bytes differ from the block already there (repeated solves of one shape reuse it; the input
  // matrix, the output and the record pointer go by value).  No-allocation calls share their scratch with
  // other contexts on the device, so they always copy.  The kernel writes its result record straight into
  // the pinned scalars, whose status slot holds a marker until the record arrives; both pinned areas
  // serve one call at a time (the call ends synchronised).
  // Only the block up to the program's last phase is uploaded and copied by the kernel.
  static_assert(((sizeof(SmParams<T>) + 15) / 16) * 16 <= Ctx::kStageBytes, "staging area");
  static_assert(S_COUNT <= 48, "pinned scalars");
  constexpr double kNoRecord = -1.0e300;
  const size_t pbytes = ((offsetof(SmParams<T>, gp) + sizeof(P.gp[0]) * prog.nphase + 15) / 16) * 16;
  auto* Pd = static_cast<SmParams<T>*>(c.ws.get("smParams", ((sizeof(SmParams<T>) + 15) / 16) * 16));
  call.pwords = (int)(pbytes / 16);
  std::memset(c.hstage, 0, pbytes);
  std::memcpy(c.hstage, &P, std::min(pbytes, sizeof(P)));
  if (c.no_alloc || c.small_params_dev != Pd || c.small_params.size() != pbytes ||
      std::memcmp(c.small_params.data(), c.hstage, pbytes) != 0) {
    QP_HIP(hipMemcpyAsync(Pd, c.hstage, pbytes, hipMemcpyHostToDevice, s));
    c.small_params.assign(static_cast<const unsigned char*>(c.hstage), static_cast<const unsigned char*>(c.hstage) + pbytes);
    c.small_params_dev = c.no_alloc ? nullptr : Pd;
  }
  call.hres = c.hsc;
  call.bar_base = c.small_bar_base;
  c.hsc[S_STATUS] = kNoRecord;
  launch_small<T>(Pd, call, grid, s);
  QP_HIP(hipStreamSynchronize(s));
  double st[S_COUNT];
  std::memcpy(st, c.hsc, sizeof(st));
  if (P.trace) {
    std::vector<unsigned long long> tr(kTrace);
    QP_HIP(hipMemcpy(tr.data(), P.trace, sizeof(unsigned long long) * kTrace, hipMemcpyDeviceToHost));
    fprintf(stderr, "[qpinv] small solve, grid %d: barrier times (us from start):", grid);
    for (int i = 1; i < kTrace && tr[i] > tr[0] && tr[i] - tr[0] < 1000000000ull; ++i)
      fprintf(stderr, " %.1f", (tr[i] - tr[0]) * 0.01);
    fprintf(stderr, "\n");
  }
  if (st[S_STATUS] == kNoRecord || st[S_GIVEUP] != 0.0) {
    // every workgroup left at a barrier whose wait expired (the give-up flag is set): the barrier words are
    // cleared before the next solve
    unsigned int barw[4];
    QP_HIP(hipMemcpy(barw, P.bar, sizeof(barw), hipMemcpyDeviceToHost));
    c.small_state = nullptr;
    if (barw[2] != 0u || st[S_GIVEUP] != 0.0) throw Error(QPINV_ETIMEOUT, "small solve: a grid barrier wait expired");
    throw Error(QPINV_EHIP, "small solve: the kernel left no result record");
  }
  c.small_bar_base = call.bar_base + (unsigned int)st[S_BARS] * (unsigned int)grid;
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
  inf.gemm_flops = inf.iters * program_flops(prog, m, n, left, e1 && inf.iters > 1, SM_MAXPH);
  if (e1 && inf.iters > 0) inf.gemm_flops += program_flops(prog, m, n, left, true, prog.e1_phase);
  c.flops += inf.gemm_flops;
  if (!direct) {
    const Mat Xr = mat_of(P.buf[1 + (int)st[S_RETBUF]], dtype);
    sm_convert(Xr, Xout, s);
    QP_HIP(hipStreamSynchronize(s));
  }
  return status;
}

}  // namespace

bool small_eligible(const Ctx& c, int method, int order, int scaling, int stop, int precision, int64_t m, int64_t n) {
  if (!c.opt.small_path || c.opt.gemm_timing || c.opt.penrose_finish) return false;
  for (int k = 0; k < 3; ++k)
    if (c.opt.force_cfg[k] >= 0) return false;
  if (precision != QPINV_PREC_F64 && precision != QPINV_PREC_F32) return false;
  if (method == QPINV_QRAPID) {
    if (qrapid_phases(order, true) > SM_MAXPH || qrapid_phases(order, false) > SM_MAXPH) return false;
  } else if (method != QPINV_NS && method != QPINV_QSAI && method != QPINV_QHPI19) {
    return false;
  }
  if (stop != STOP_DX_ABS && stop != STOP_DX_REL && stop != STOP_E1_REL) return false;
  if (scaling != QPINV_ALPHA_POWER && scaling != QPINV_ALPHA_FROB && scaling != QPINV_ALPHA_GIVEN) return false;
  return m >= 1 && n >= 1 && m <= SM_MAXD && n <= SM_MAXD;
}

int small_solve(Ctx& c, int method, int order, const Mat& A0, int scaling, double am, double tol, int max_iter,
                int stop, int precision, const Mat& Xout, qpinv_info& inf, hipStream_t s) {
  if (precision == QPINV_PREC_F64)
    return small_solve_t<double>(c, method, order, A0, scaling, am, tol, max_iter, stop, QPINV_F64, Xout, inf, s);
  return small_solve_t<float>(c, method, order, A0, scaling, am, tol, max_iter, stop, QPINV_F32, Xout, inf, s);
}

}  // namespace qp

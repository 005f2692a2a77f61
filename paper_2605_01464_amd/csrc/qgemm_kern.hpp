// Device-side pieces shared by the quaternion GEMM kernels (FP32/FP64 and BF16 variants).
#pragma once

#include "qgemm.hpp"

namespace qp {

// ------------------------------------------------------------------------------------------------
// MFMA shapes.  Lane layouts (64 lanes):
//   32x32x2 f32 : A frag  A[i = l%32][k = l/32], B frag B[k = l/32][j = l%32],
//                 D reg r: row 8(r/4) + 4(l/32) + r%4, col l%32
//   16x16x4 f32 : A[i = l%16][k = l/16], B[k = l/16][j = l%16], D reg r: row 4(l/16) + r, col l%16
//   16x16x4 f64 : same A and B, D reg r (one double): row l/16 + 4r, col l%16
// ------------------------------------------------------------------------------------------------
struct MM32F {
  using T = float;
  using Acc = floatx16;
  static constexpr int BLK = 32, KS = 2, NR = 16;
  __device__ static int fr(int l) { return l & 31; }
  __device__ static int fk(int l) { return l >> 5; }
  __device__ static int crow(int l, int r) { return ((r >> 2) << 3) + ((l >> 5) << 2) + (r & 3); }
  __device__ static int ccol(int l) { return l & 31; }
  __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
};

struct MM16F {
  using T = float;
  using Acc = floatx4;
  static constexpr int BLK = 16, KS = 4, NR = 4;
  __device__ static int fr(int l) { return l & 15; }
  __device__ static int fk(int l) { return l >> 4; }
  __device__ static int crow(int l, int r) { return ((l >> 4) << 2) + r; }
  __device__ static int ccol(int l) { return l & 15; }
  __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

struct MM16D {
  using T = double;
  using Acc = doublex4;
  static constexpr int BLK = 16, KS = 4, NR = 4;
  __device__ static int fr(int l) { return l & 15; }
  __device__ static int fk(int l) { return l >> 4; }
  __device__ static int crow(int l, int r) { return (l >> 4) + (r << 2); }
  __device__ static int ccol(int l) { return l & 15; }
  __device__ static Acc mma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

template <class T>
struct V16;
typedef double doublex2 __attribute__((ext_vector_type(2)));
template <>
struct V16<float> {
  using type = float4;
  using nat = floatx4;  // the native vector type, for loads through address space 1
  static constexpr int n = 4;
};
template <>
struct V16<double> {
  using type = double2;
  using nat = doublex2;
  static constexpr int n = 2;
};

template <class T>
struct GemmParams {
  const T* A;
  int64_t lda, psa;
  const T* B;
  int64_t ldb, psb;
  int M, N, K;
  int tiles_m, tiles_n;
  int vec;  // 16-byte vector loads allowed (aligned bases, ld and plane strides)
  int nout, nin, ref;
  T* out[3];
  int64_t ldo[3], pso[3];
  const T* in[3];
  int64_t ldi[3], psi[3];
  T ca[3], cb[3][3], cg[3];
  double* partial;  // per-workgroup partial sums of the reduction (standalone kernels)
  int reduce;       // accumulate the reduction terms
};

// Global-memory accesses through address space 1.  A pointer that was loaded from memory (a batch
// descriptor) or passed through readfirstlane is generic to the compiler, and generic (flat) accesses
// count against the LDS wait counter too, so every LDS wait would also wait for loads in flight.
template <class T>
__device__ __forceinline__ T gload(const T* p, int64_t i) {
  return ((const __attribute__((address_space(1))) T*)p)[i];
}
template <class T>
__device__ __forceinline__ void gstore(T* p, int64_t i, T v) {
  ((__attribute__((address_space(1))) T*)p)[i] = v;
}

// Hamilton product of one fragment set: acc_p += sum_q sign(p,q) a_q b_{r(p,q)}.
template <class MM>
__device__ __forceinline__ void quat_mma(typename MM::Acc (&acc)[4], const typename MM::T (&a)[4],
                                         const typename MM::T (&b)[4]) {
  const auto na1 = -a[1], na2 = -a[2], na3 = -a[3];
  acc[0] = MM::mma(a[0], b[0], acc[0]);
  acc[0] = MM::mma(na1, b[1], acc[0]);
  acc[0] = MM::mma(na2, b[2], acc[0]);
  acc[0] = MM::mma(na3, b[3], acc[0]);
  acc[1] = MM::mma(a[0], b[1], acc[1]);
  acc[1] = MM::mma(a[1], b[0], acc[1]);
  acc[1] = MM::mma(a[2], b[3], acc[1]);
  acc[1] = MM::mma(na3, b[2], acc[1]);
  acc[2] = MM::mma(a[0], b[2], acc[2]);
  acc[2] = MM::mma(na1, b[3], acc[2]);
  acc[2] = MM::mma(a[2], b[0], acc[2]);
  acc[2] = MM::mma(a[3], b[1], acc[2]);
  acc[3] = MM::mma(a[0], b[3], acc[3]);
  acc[3] = MM::mma(a[1], b[2], acc[3]);
  acc[3] = MM::mma(na2, b[1], acc[3]);
  acc[3] = MM::mma(a[3], b[0], acc[3]);
}

__device__ __forceinline__ void tile_of_block(int bid, int nb, int tiles_m, int tiles_n, int& tm, int& tn) {
  if ((nb & 7) == 0) {
    const int per = nb >> 3;
    bid = (bid & 7) * per + (bid >> 3);
  }
  constexpr int GM = 8;
  const int width = GM * tiles_n;
  const int group = bid / width;
  const int first = group * GM;
  const int gs = min(tiles_m - first, GM);
  const int in_group = bid - group * width;
  tm = first + in_group % gs;
  tn = in_group / gs;
}


// The epilogue inputs in_u of plane p at one element (0 outside the output or beyond nin).
template <class T>
__device__ __forceinline__ void epilogue_inputs(const GemmParams<T>& P, int p, int row, int col, T (&inv)[3]) {
  // the load address is clamped into the matrix and the value selected afterwards: no branch per load
  const bool ok = row < P.M && col < P.N;
  const int64_t r = row < P.M ? row : P.M - 1, c = col < P.N ? col : P.N - 1;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    if (u < P.nin) {
      const T x = gload(P.in[u], p * P.psi[u] + r * P.ldi[u] + c);
      inv[u] = ok ? x : T(0);
    } else {
      inv[u] = T(0);
    }
  }
}

// The same inputs with every load issued before any is used: all three loads go out without a branch on
// the input count (an absent input re-reads a valid address: the first input's element, or the first
// element of A) and the values are selected afterwards.  Under a branch each load is waited for inside
// it, one memory latency per load; this form costs one latency for all of them, at the price of more
// scalar registers (for latency-bound tiles: the batched and one-launch solvers).
template <class T>
__device__ __forceinline__ void epilogue_inputs_overlap(const GemmParams<T>& P, int p, int row, int col, T (&inv)[3]) {
  const bool ok = row < P.M && col < P.N;
  const int64_t r = row < P.M ? row : P.M - 1, c = col < P.N ? col : P.N - 1;
  const bool any = P.nin > 0;
  const T* const base = any ? P.in[0] : P.A;
  const int64_t off0 = any ? p * P.psi[0] + r * P.ldi[0] + c : 0;
  T x[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const bool use = u < P.nin;
    x[u] = gload(use ? P.in[u] : base, use ? p * P.psi[u] + r * P.ldi[u] + c : off0);
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) inv[u] = ok && u < P.nin ? x[u] : T(0);
}

// out_t = a_t v + sum_u b_tu in_u + g_t I for plane p at one element, plus the reduction terms; inv
// holds the element's inputs (epilogue_inputs).
template <class T>
__device__ __forceinline__ void epilogue_apply(const GemmParams<T>& P, int p, int row, int col, T v, const T (&inv)[3],
                                               double& s_d, double& s_x) {
  if (row >= P.M || col >= P.N) return;
  const T eye = (p == 0 && row == col) ? T(1) : T(0);
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t < P.nout) {
      const T o = P.ca[t] * v + P.cg[t] * eye + P.cb[t][0] * inv[0] + P.cb[t][1] * inv[1] + P.cb[t][2] * inv[2];
      gstore(P.out[t], p * P.pso[t] + (int64_t)row * P.ldo[t] + col, o);
      if (t == 0 && P.reduce) {
        const double od = (double)o;
        const double ref = P.ref == 0 ? (double)inv[0] : P.ref == 1 ? (double)inv[1] : P.ref == 2 ? (double)inv[2] : 0.0;
        const double dd = od - ref;
        s_d += dd * dd;
        s_x += od * od;
      }
    }
  }
}

// Workgroup sum of the epilogue reduction terms, written to partial[2 * blockIdx.x + {0, 1}].
template <int NW>
__device__ __forceinline__ void store_partials(double* partial, double s_d, double s_x, double (*red_lds)[2], int lane,
                                               int w, int tid) {
  if (!partial) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s_d += __shfl_xor(s_d, off, 64);
    s_x += __shfl_xor(s_x, off, 64);
  }
  if (lane == 0) {
    red_lds[w][0] = s_d;
    red_lds[w][1] = s_x;
  }
  __syncthreads();
  if (tid == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int q = 0; q < NW; ++q) {
      a0 += red_lds[q][0];
      a1 += red_lds[q][1];
    }
    partial[2 * (int64_t)blockIdx.x] = a0;
    partial[2 * (int64_t)blockIdx.x + 1] = a1;
  }
}

template <class MM, int BM, int BN, int BK, int WM, int WN>
struct GemmCfg {
  using T = typename MM::T;
  static constexpr int NW = WM * WN, NT = 64 * NW;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / MM::BLK, TN = WTN / MM::BLK;
  static constexpr int PADB = (sizeof(T) == 4) ? 4 : 2;
  static constexpr int LDB = BN + PADB;
  static constexpr int VA = V16<T>::n;
  // A staging: [plane][k chunk of VA][row, BM + 2 rows of padding][VA]; the padding puts the four
  // chunks a group of lanes writes (consecutive k chunks of two rows) and reads on distinct banks.
  static constexpr int LDAC = BM + 2;
  static constexpr int KB = VA * MM::KS;  // k covered by one 16-byte fragment read (VA MFMAs)
  static constexpr int AELEMS = 4 * (BK / VA) * LDAC * VA;
  static constexpr int ACH = BM * BK / VA;  // 16-byte chunks per plane of an A tile
  static constexpr int BCH = BK * BN / VA;
  static constexpr int NA = (ACH + NT - 1) / NT;
  static constexpr int NB = (BCH + NT - 1) / NT;
  static_assert(TM >= 1 && TN >= 1 && WTM % MM::BLK == 0 && WTN % MM::BLK == 0, "wave tile");
  static_assert(BK % KB == 0 && BN % VA == 0, "k tile");
  static constexpr int SMEM = AELEMS + 4 * BK * LDB;  // elements of T (one staging buffer)
  static constexpr size_t LDS_BYTES = sizeof(T) * SMEM;
  static_assert(LDS_BYTES <= 65536, "LDS budget");
};

// Operand load modes of gemm_tile.
//   kLoadScalar:  any ld; tiles that cross the matrix edge load element by element.
//   kLoadVec:     16-byte aligned bases, ld and plane strides (GemmParams::vec); edge tiles take the same
//                 16-byte loads from a row and a k chunk clamped into the matrix.  A row may then be
//                 read up to ld (never past it), and the elements outside the matrix are replaced by
//                 zeros: any value there, NaN included, leaves the product unchanged.
//   kLoadAligned: kLoadVec, and M % BM = N % BN = K % BK = 0: no clamps and no masks.
enum : int { kLoadScalar = 0, kLoadVec = 1, kLoadAligned = 2 };

// One BM x BN output tile (all four planes) of C = A B with the epilogue; the epilogue's reduction
// terms are added to the caller's s_d, s_x.  Used by the standalone product kernel and by the batched
// solver (a workgroup walks all tiles).
//   LM:      the operand load mode (above).
//   DB:      two LDS staging buffers (`smem` holds 2 C::SMEM elements): the next K step is written to
//            one while the MFMAs read the other, one barrier per K step; otherwise one buffer
//            (C::SMEM elements) and two barriers per K step.
//   OVL:     the epilogue's inputs loaded by epilogue_inputs_overlap (all loads in flight together).
template <class MM, int BM, int BN, int BK, int WM, int WN, int FLUSH, int LM = kLoadScalar, bool DB = false,
          bool OVL = false>
__device__ __forceinline__ void gemm_tile(const GemmParams<typename MM::T>& P, int tm, int tn, typename MM::T* smem,
                                          double& s_d, double& s_x) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  using T = typename MM::T;
  using Acc = typename MM::Acc;
  using VT = typename V16<T>::type;
  constexpr int VA = C::VA;
  static_assert(FLUSH == 0 || FLUSH % BK == 0, "flush interval is a whole number of K tiles");
  static_assert(MM::NR <= 4 || C::NW * MM::BLK * MM::BLK <= C::SMEM, "epilogue slabs fit in the staging LDS");

  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wm = w % WM, wn = w / WM;

  Acc acc[4][C::TM][C::TN];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
#pragma unroll
        for (int r = 0; r < MM::NR; ++r) acc[p][i][j][r] = T(0);

  // Two-level accumulation: the MFMA accumulators cover FLUSH consecutive k and are then added into
  // `tot`, so no FP32 rounding chain is longer than FLUSH/KS + K/FLUSH additions.
  constexpr int TT = FLUSH > 0 ? 4 : 1;  // a 1-element placeholder when the flush is off
  Acc tot[TT][FLUSH > 0 ? C::TM : 1][FLUSH > 0 ? C::TN : 1];
  if constexpr (FLUSH > 0) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j)
#pragma unroll
          for (int r = 0; r < MM::NR; ++r) tot[p][i][j][r] = T(0);
  }
  auto flush = [&]() {
    if constexpr (FLUSH > 0) {
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
          for (int j = 0; j < C::TN; ++j)
#pragma unroll
            for (int r = 0; r < MM::NR; ++r) {
              tot[p][i][j][r] += acc[p][i][j][r];
              acc[p][i][j][r] = T(0);
            }
    }
  };

  T ra[4][C::NA][VA];
  T rb[4][C::NB][VA];

  // Edge tiles in kLoadScalar mode load every element from an address clamped into the matrix; in
  // kLoadVec mode the 16-byte chunk is clamped.  Either way the elements outside the matrix are zeroed
  // only when the registers go to LDS, so the loads stay in flight behind the MFMAs like full-tile ones.
  constexpr bool ALIGNED = LM == kLoadAligned;
  auto full_a = [&](int k0) { return ALIGNED || (LM == kLoadVec && (m0 + BM <= P.M) && (k0 + BK <= P.K)); };
  auto full_b = [&](int k0) { return ALIGNED || (LM == kLoadVec && (n0 + BN <= P.N) && (k0 + BK <= P.K)); };
  using VG = typename V16<T>::nat;
  // last chunk start that holds an element of the matrix (kLoadVec): k chunks of A, column chunks of B
  const int kc_last = ((P.K - 1) / VA) * VA, jc_last = ((P.N - 1) / VA) * VA;
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T* Aq = P.A + q * P.psa;
#pragma unroll
      for (int t = 0; t < C::NA; ++t) {
        const int c = tid + t * C::NT;
        const int i = c / (BK / VA), kc = (c % (BK / VA)) * VA;
        if (C::ACH % C::NT == 0 || c < C::ACH) {
          const int gi = m0 + i, gk = k0 + kc;
          if constexpr (LM == kLoadScalar) {
            const int64_t ci = gi < P.M ? gi : P.M - 1;
#pragma unroll
            for (int e = 0; e < VA; ++e) ra[q][t][e] = gload(Aq, ci * P.lda + (gk + e < P.K ? gk + e : P.K - 1));
          } else {
            const int64_t ci = ALIGNED || gi < P.M ? gi : P.M - 1;
            const int ck = ALIGNED || gk <= kc_last ? gk : kc_last;
            const VG v = gload(reinterpret_cast<const VG*>(Aq + ci * P.lda + ck), 0);
#pragma unroll
            for (int e = 0; e < VA; ++e) ra[q][t][e] = v[e];
          }
        }
      }
      const T* Bq = P.B + q * P.psb;
#pragma unroll
      for (int t = 0; t < C::NB; ++t) {
        const int c = tid + t * C::NT;
        const int k = c / (BN / VA), jc = (c % (BN / VA)) * VA;
        if (C::BCH % C::NT == 0 || c < C::BCH) {
          const int gk = k0 + k, gj = n0 + jc;
          if constexpr (LM == kLoadScalar) {
            const int64_t ck = gk < P.K ? gk : P.K - 1;
#pragma unroll
            for (int e = 0; e < VA; ++e) rb[q][t][e] = gload(Bq, ck * P.ldb + (gj + e < P.N ? gj + e : P.N - 1));
          } else {
            const int64_t ck = ALIGNED || gk < P.K ? gk : P.K - 1;
            const int cj = ALIGNED || gj <= jc_last ? gj : jc_last;
            const VG v = gload(reinterpret_cast<const VG*>(Bq + ck * P.ldb + cj), 0);
#pragma unroll
            for (int e = 0; e < VA; ++e) rb[q][t][e] = v[e];
          }
        }
      }
    }
  };

  // registers of K step k0 to LDS
  auto store = [&](T* As, T* Bs, int k0) {
    const bool fullA = full_a(k0), fullB = full_b(k0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int t = 0; t < C::NA; ++t) {
        const int c = tid + t * C::NT;
        if (C::ACH % C::NT == 0 || c < C::ACH) {
          const int i = c / (BK / VA), kc = (c % (BK / VA)) * VA;
          const bool rin = m0 + i < P.M;
          VT v;
          T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
          for (int e = 0; e < VA; ++e) pv[e] = (fullA || (rin && k0 + kc + e < P.K)) ? ra[q][t][e] : T(0);
          *reinterpret_cast<VT*>(&As[((q * (BK / VA) + kc / VA) * C::LDAC + i) * VA]) = v;
        }
      }
#pragma unroll
      for (int t = 0; t < C::NB; ++t) {
        const int c = tid + t * C::NT;
        if (C::BCH % C::NT == 0 || c < C::BCH) {
          const int k = c / (BN / VA), jc = (c % (BN / VA)) * VA;
          const bool kin = k0 + k < P.K;
          VT v;
          T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
          for (int e = 0; e < VA; ++e) pv[e] = (fullB || (kin && n0 + jc + e < P.N)) ? rb[q][t][e] : T(0);
          *reinterpret_cast<VT*>(&Bs[(q * BK + k) * C::LDB + jc]) = v;
        }
      }
    }
  };

  // MFMA k-group g = fk(lane) of a block of KB k takes the VA consecutive k of chunk g from one 16-byte
  // LDS read; the e-th of the block's VA MFMAs uses element e of every lane (k = VA g + e), so the VA
  // MFMAs together sum the block's KB products (in a different order than k = 0, 1, ...).
  const int fr = MM::fr(lane), fk = MM::fk(lane);
  auto compute = [&](const T* As, const T* Bs) {
#pragma unroll
    for (int kb = 0; kb < BK / C::KB; ++kb) {
      VT av[C::TM][4];
      T b[C::TN][4][VA];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
          av[i][q] = *reinterpret_cast<const VT*>(
              &As[((q * (BK / VA) + kb * MM::KS + fk) * C::LDAC + wm * C::WTM + i * MM::BLK + fr) * VA]);
#pragma unroll
        for (int j = 0; j < C::TN; ++j)
#pragma unroll
          for (int e = 0; e < VA; ++e)
            b[j][q][e] = Bs[(q * BK + kb * C::KB + VA * fk + e) * C::LDB + wn * C::WTN + j * MM::BLK + fr];
      }
#pragma unroll
      for (int e = 0; e < VA; ++e)
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
          for (int j = 0; j < C::TN; ++j) {
            T a4[4], b4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              a4[q] = reinterpret_cast<const T*>(&av[i][q])[e];
              b4[q] = b[j][q][e];
            }
            Acc t4[4] = {acc[0][i][j], acc[1][i][j], acc[2][i][j], acc[3][i][j]};
            quat_mma<MM>(t4, a4, b4);
#pragma unroll
            for (int p = 0; p < 4; ++p) acc[p][i][j] = t4[p];
          }
    }
  };
  constexpr int BOFF = C::AELEMS;  // B staging follows A staging in a buffer
  if constexpr (!DB) {
    if (P.K > 0) load(0);
    for (int k0 = 0; k0 < P.K; k0 += BK) {
      __syncthreads();
      store(smem, smem + BOFF, k0);
      __syncthreads();
      if (k0 + BK < P.K) load(k0 + BK);
      compute(smem, smem + BOFF);
      if constexpr (FLUSH > 0) {
        if ((k0 + BK) % FLUSH == 0) flush();
      }
    }
  } else {
    // buffer b holds K step s with s % 2 == b.  Step s reads buffer s % 2 while step s + 1 is written
    // to the other one (whose last reader was step s - 1, behind the previous barrier) and step s + 2
    // is fetched into registers.
    __syncthreads();  // the caller may have used the LDS just before (previous tile's epilogue)
    if (P.K > 0) {
      load(0);
      store(smem, smem + BOFF, 0);
      if (BK < P.K) load(BK);
    }
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < P.K; k0 += BK) {
      T* const Ac = smem + cur * C::SMEM;
      compute(Ac, Ac + BOFF);
      if (k0 + BK < P.K) {
        T* const An = smem + (cur ^ 1) * C::SMEM;
        store(An, An + BOFF, k0 + BK);
        if (k0 + 2 * BK < P.K) load(k0 + 2 * BK);
      }
      if constexpr (FLUSH > 0) {
        if ((k0 + BK) % FLUSH == 0) flush();
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  flush();

  // ---------------------------------------------------------------- epilogue
  // Register r of a lane holds element (crow(lane, r), ccol(lane)) of its MFMA block.  With 4 registers
  // per block (16 x 16 MFMA) the outputs go straight from the accumulators: a store instruction writes
  // 16-element row segments, as coalesced as a pass through LDS would be, without its barriers.  With
  // 16 (32 x 32 MFMA) each block goes through a per-wave LDS slab first, which keeps the accumulators
  // read with compile-time indices and the register count at the K loop's.  Either way the inputs of
  // up to 4 elements are loaded first (one memory latency per group), then their outputs written.
  constexpr int NE = MM::BLK * MM::BLK / 64, NG = NE < 4 ? NE : 4;
  auto value = [&](int p, int i, int j, int r) -> T {
    if constexpr (FLUSH > 0)
      return tot[p][i][j][r];
    else
      return acc[p][i][j][r];
  };
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int rb = m0 + wm * C::WTM + i * MM::BLK, cb = n0 + wn * C::WTN + j * MM::BLK;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if constexpr (MM::NR <= 4) {
          T inv[MM::NR][3];
#pragma unroll
          for (int r = 0; r < MM::NR; ++r) {
            if constexpr (OVL)
              epilogue_inputs_overlap(P, p, rb + MM::crow(lane, r), cb + MM::ccol(lane), inv[r]);
            else
              epilogue_inputs(P, p, rb + MM::crow(lane, r), cb + MM::ccol(lane), inv[r]);
          }
#pragma unroll
          for (int r = 0; r < MM::NR; ++r)
            epilogue_apply(P, p, rb + MM::crow(lane, r), cb + MM::ccol(lane), value(p, i, j, r), inv[r], s_d, s_x);
        } else {
          T* const slab = smem + w * MM::BLK * MM::BLK;
          __syncthreads();
#pragma unroll
          for (int r = 0; r < MM::NR; ++r) slab[MM::crow(lane, r) * MM::BLK + MM::ccol(lane)] = value(p, i, j, r);
          __syncthreads();
          for (int k0 = 0; k0 < NE; k0 += NG) {
            T inv[NG][3];
#pragma unroll
            for (int k = 0; k < NG; ++k) {
              const int e = lane + 64 * (k0 + k);
              if constexpr (OVL)
                epilogue_inputs_overlap(P, p, rb + e / MM::BLK, cb + e % MM::BLK, inv[k]);
              else
                epilogue_inputs(P, p, rb + e / MM::BLK, cb + e % MM::BLK, inv[k]);
            }
#pragma unroll
            for (int k = 0; k < NG; ++k) {
              const int e = lane + 64 * (k0 + k);
              epilogue_apply(P, p, rb + e / MM::BLK, cb + e % MM::BLK, slab[e], inv[k], s_d, s_x);
            }
          }
        }
      }
    }
  __syncthreads();  // the staging LDS is reused by whatever runs next in this workgroup
}


}  // namespace qp

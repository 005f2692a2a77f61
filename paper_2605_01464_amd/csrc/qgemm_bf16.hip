// Quaternion GEMM with BF16 operands on gfx950 MFMA (v_mfma_f32_16x16x32_bf16), FP32 storage and
// FP32 accumulation: the early, self-correcting iterations of the precision ladder.
//
// The operand planes stay FP32 in HBM; each workgroup rounds them to BF16 (round to nearest even)
// while staging into LDS, so no BF16 copy of any matrix exists.  Two forms: a single-buffered one
// (small tiles) and a double-buffered one (below).  Fragment lane layout of the MFMA (64 lanes):
//   A frag: row l%16, k = 8(l/16) .. 8(l/16)+7;  B frag: col l%16, same k;  D reg r: row 4(l/16)+r, col l%16.
#include <algorithm>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "qgemm_kern.hpp"

namespace qp {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 neg_bf16x8(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ floatx4 mma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Single-buffered form.  LDS holds A tiles as [plane][row][k] and B tiles transposed as [plane][col][k],
// both k-contiguous with 8 elements of row padding, so that every lane reads its eight consecutive k
// of a fragment with one 16-byte LDS load.
template <int BM, int BN, int WM, int WN>
struct Bf16Cfg {
  static constexpr int BK = 32, BLK = 16, NR = 4;
  static constexpr int NW = WM * WN, NT = 64 * NW;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / BLK, TN = WTN / BLK;
  static constexpr int LDK = BK + 8;  // bf16 elements per LDS row (80 bytes: 16-byte aligned rows)
  static constexpr int ACH = BM * BK / 4, BCH = BN * BK / 4;  // 4-element chunks per plane
  static constexpr int NA = (ACH + NT - 1) / NT, NB = (BCH + NT - 1) / NT;
  static constexpr size_t LDS = 2 * 4 * (BM + BN) * LDK;
  static_assert(TM >= 1 && TN >= 1 && WTM % BLK == 0 && WTN % BLK == 0, "wave tile");
  static_assert(LDS <= 65536, "LDS budget");
  static_assert(NW * BLK * BLK * 4 <= (int)LDS, "epilogue staging fits");
};

// One BM x BN output tile (all four planes) with the epilogue; adds the reduction terms to s_d, s_x.
template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void bf16_tile(const GemmParams<float>& P, int tm, int tn, __bf16* smem, double& s_d,
                                          double& s_x) {
  using C = Bf16Cfg<BM, BN, WM, WN>;
  constexpr int BK = C::BK, LDK = C::LDK;
  __bf16* const As = smem;                 // [4][BM][LDK]
  __bf16* const Bs = smem + 4 * BM * LDK;  // [4][BN][LDK]
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w % WM, wn = w / WM;

  floatx4 acc[4][C::TM][C::TN];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) acc[p][i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  float ra[4][C::NA][4], rb[4][C::NB][4];

  // A chunk c: row i = c / (BK/4), k = 4 (c % (BK/4)) .. +3 (one 16-byte global load).
  // B chunk c: col j = c % BN, k = 4 (c / BN) .. +3 (four loads, each coalesced across the wave).
  auto load = [&](int k0) {
    const bool fullA = P.vec && (m0 + BM <= P.M) && (k0 + BK <= P.K);
    const bool fullB = (n0 + BN <= P.N) && (k0 + BK <= P.K);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float* Aq = P.A + q * P.psa;
#pragma unroll
      for (int t = 0; t < C::NA; ++t) {
        const int c = tid + t * C::NT;
        if (C::ACH % C::NT == 0 || c < C::ACH) {
          const int gi = m0 + c / (BK / 4), gk = k0 + (c % (BK / 4)) * 4;
          if (fullA) {
            const float4 v = *reinterpret_cast<const float4*>(Aq + (int64_t)gi * P.lda + gk);
            ra[q][t][0] = v.x;
            ra[q][t][1] = v.y;
            ra[q][t][2] = v.z;
            ra[q][t][3] = v.w;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              ra[q][t][e] = (gi < P.M && gk + e < P.K) ? Aq[(int64_t)gi * P.lda + gk + e] : 0.f;
          }
        }
      }
      const float* Bq = P.B + q * P.psb;
#pragma unroll
      for (int t = 0; t < C::NB; ++t) {
        const int c = tid + t * C::NT;
        if (C::BCH % C::NT == 0 || c < C::BCH) {
          const int gj = n0 + c % BN, gk = k0 + (c / BN) * 4;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            rb[q][t][e] = (fullB || (gj < P.N && gk + e < P.K)) ? Bq[(int64_t)(gk + e) * P.ldb + gj] : 0.f;
        }
      }
    }
  };

  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int t = 0; t < C::NA; ++t) {
        const int c = tid + t * C::NT;
        if (C::ACH % C::NT == 0 || c < C::ACH) {
          const int i = c / (BK / 4), kc = (c % (BK / 4)) * 4;
          const bf16x4 v = {(__bf16)ra[q][t][0], (__bf16)ra[q][t][1], (__bf16)ra[q][t][2], (__bf16)ra[q][t][3]};
          *reinterpret_cast<bf16x4*>(&As[(q * BM + i) * LDK + kc]) = v;
        }
      }
#pragma unroll
      for (int t = 0; t < C::NB; ++t) {
        const int c = tid + t * C::NT;
        if (C::BCH % C::NT == 0 || c < C::BCH) {
          const int j = c % BN, kc = (c / BN) * 4;
          const bf16x4 v = {(__bf16)rb[q][t][0], (__bf16)rb[q][t][1], (__bf16)rb[q][t][2], (__bf16)rb[q][t][3]};
          *reinterpret_cast<bf16x4*>(&Bs[(q * BN + j) * LDK + kc]) = v;
        }
      }
    }
  };

  const int fr = lane & 15, fk = (lane >> 4) * 8;
  if (P.K > 0) load(0);
  for (int k0 = 0; k0 < P.K; k0 += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + BK < P.K) load(k0 + BK);
    bf16x8 a[C::TM][4], b[C::TN][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
        a[i][q] = *reinterpret_cast<const bf16x8*>(&As[(q * BM + wm * C::WTM + i * 16 + fr) * LDK + fk]);
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
        b[j][q] = *reinterpret_cast<const bf16x8*>(&Bs[(q * BN + wn * C::WTN + j * 16 + fr) * LDK + fk]);
    }
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      const bf16x8 na1 = neg_bf16x8(a[i][1]), na2 = neg_bf16x8(a[i][2]), na3 = neg_bf16x8(a[i][3]);
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        // Hamilton product: acc_p += sum_q sign(p, q) a_q b_{r(p, q)}
        acc[0][i][j] = mma_bf16(a[i][0], b[j][0], acc[0][i][j]);
        acc[0][i][j] = mma_bf16(na1, b[j][1], acc[0][i][j]);
        acc[0][i][j] = mma_bf16(na2, b[j][2], acc[0][i][j]);
        acc[0][i][j] = mma_bf16(na3, b[j][3], acc[0][i][j]);
        acc[1][i][j] = mma_bf16(a[i][0], b[j][1], acc[1][i][j]);
        acc[1][i][j] = mma_bf16(a[i][1], b[j][0], acc[1][i][j]);
        acc[1][i][j] = mma_bf16(a[i][2], b[j][3], acc[1][i][j]);
        acc[1][i][j] = mma_bf16(na3, b[j][2], acc[1][i][j]);
        acc[2][i][j] = mma_bf16(a[i][0], b[j][2], acc[2][i][j]);
        acc[2][i][j] = mma_bf16(na1, b[j][3], acc[2][i][j]);
        acc[2][i][j] = mma_bf16(a[i][2], b[j][0], acc[2][i][j]);
        acc[2][i][j] = mma_bf16(a[i][3], b[j][1], acc[2][i][j]);
        acc[3][i][j] = mma_bf16(a[i][0], b[j][3], acc[3][i][j]);
        acc[3][i][j] = mma_bf16(a[i][1], b[j][2], acc[3][i][j]);
        acc[3][i][j] = mma_bf16(na2, b[j][1], acc[3][i][j]);
        acc[3][i][j] = mma_bf16(a[i][3], b[j][0], acc[3][i][j]);
      }
    }
  }

  // epilogue through a per-wave FP32 slab (static accumulator indices, row-contiguous output pass)
  float* const slab = reinterpret_cast<float*>(smem) + w * 16 * 16;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j)
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) slab[(((lane >> 4) << 2) + r) * 16 + (lane & 15)] = acc[p][i][j][r];
        __syncthreads();
        const int rb0 = m0 + wm * C::WTM + i * 16, cb0 = n0 + wn * C::WTN + j * 16;
        float inv[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int e = lane + 64 * k;
          epilogue_inputs(P, p, rb0 + e / 16, cb0 + e % 16, inv[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int e = lane + 64 * k;
          epilogue_apply(P, p, rb0 + e / 16, cb0 + e % 16, slab[e], inv[k], s_d, s_x);
        }
      }
  __syncthreads();  // LDS is reused by the workgroup's next tile
}

// Tiles blockIdx.x, blockIdx.x + gridDim.x, ... (one tile when the grid covers them all).
template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) qgemm_bf16_kernel(GemmParams<float> P) {
  using C = Bf16Cfg<BM, BN, WM, WN>;
  __shared__ __attribute__((aligned(16))) __bf16 smem[4 * (BM + BN) * C::LDK];
  __shared__ double red_lds[C::NW][2];
  const int nt = P.tiles_m * P.tiles_n;
  double s_d = 0.0, s_x = 0.0;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int tm, tn;
    tile_of_block(t, nt, P.tiles_m, P.tiles_n, tm, tn);
    bf16_tile<BM, BN, WM, WN>(P, tm, tn, smem, s_d, s_x);
  }
  store_partials<C::NW>(P.partial, s_d, s_x, red_lds, threadIdx.x & 63, threadIdx.x >> 6, threadIdx.x);
}

// ---------------------------------------------------------------------------------------------------
// Double-buffered form.  Per K step (32) a workgroup fetches the FP32 A tile as 16-byte row chunks and
// the FP32 B tile as 2 x 4 blocks (two 16-byte row loads, regrouped in registers to k-pairs of one
// column), rounds to BF16 (packed converts) and writes the other LDS stage while the MFMAs read this
// one: one barrier per K step.  The next stage's A tile is fetched during the first half of the MFMAs
// and its B tile during the second half, so that only one of them is held in registers.
//
// LDS rows hold the 32 k of one row (A) or column (B) of one plane, 64 bytes, with the four 16-byte k
// chunks of row r permuted by (r >> 1) & 3 so that the 8 lanes of one fragment read phase hit
// distinct banks.  With 16-byte aligned operands (BUF) the loads are buffer loads over the four planes:
// the per-tile part of each address is a lane offset and the per-step part (plane, k) a scalar
// offset, so a K step spends no vector instructions on addresses.  Steps of partial tiles and the last
// partial K step take a separate path: addresses clamped into the matrix (a row's ld extent is
// readable), and what lies outside zeroed at the LDS store.  Accumulators go straight to the epilogue.
template <int BM, int BN, int WM, int WN>
struct Bf16DbCfg {
  static constexpr int BK = 32;
  static constexpr int NW = WM * WN, NT = 64 * NW;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / 16, TN = WTN / 16;
  static constexpr int JB = BN / 4;                // column blocks of a B tile
  static constexpr int ACH = BM * BK / 4;          // 4-float chunks of one A plane tile
  static constexpr int BBL = (BK / 2) * JB;        // 2 x 4 blocks of one B plane tile
  static constexpr int NA = ACH / NT, NB = BBL / NT;
  static constexpr int STAGE = 4 * (BM + BN) * BK;  // bf16 elements of one stage
  static_assert(TM >= 2 && TN >= 1 && WTM % 16 == 0 && WTN % 16 == 0, "wave tile (two row halves)");
  static_assert(ACH % NT == 0 && BBL % NT == 0 && NT % JB == 0, "whole chunks and blocks per thread");
  static_assert(2 * STAGE * 2 <= 160 * 1024, "two stages fit the LDS");
};

// bf16 element offset of (LDS row r, 16-byte k chunk c) in the permuted layout
__device__ __forceinline__ int db_off(int r, int c) { return r * 32 + ((c ^ ((r >> 1) & 3)) << 3); }

__device__ __forceinline__ floatx4 buf_load4(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

template <int BM, int BN, int WM, int WN, bool BUF>
__device__ __forceinline__ void bf16_db_tile(const GemmParams<float>& P, int tm, int tn, __bf16* smem, double& s_d,
                                             double& s_x) {
  using C = Bf16DbCfg<BM, BN, WM, WN>;
  constexpr int BK = C::BK, JB = C::JB;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w % WM, wn = w / WM;
  const int lastk = (P.K - 1) & ~3, lastn = (P.N - 1) & ~3;
  const bool full_mn = m0 + BM <= P.M && n0 + BN <= P.N;
  // A chunks of this thread: rows tid / 8 + t NT / 8, k 4 (tid % 8) .. +3.  B blocks: columns
  // 4 (tid % JB) .. +3, k rows 2 kb(t) and 2 kb(t) + 1 with kb(t) = tid / JB + t NT / JB.
  const int kqa = tid & 7, jqb = tid % JB;
  const int colb = min(n0 + 4 * jqb, lastn);
  int rowa[C::NA];
#pragma unroll
  for (int t = 0; t < C::NA; ++t) rowa[t] = min(m0 + (tid + t * C::NT) / 8, P.M - 1);
  auto kb = [&](int t) __attribute__((always_inline)) { return (tid + t * C::NT) / JB; };

  // raw buffers over the four planes (extents below 2^31 bytes, checked by the launcher when BUF)
  const __amdgpu_buffer_rsrc_t srcA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(P.A), (short)0, (int)((3 * P.psa + (int64_t)P.M * P.lda) * 4), 0x00020000);
  const __amdgpu_buffer_rsrc_t srcB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(P.B), (short)0, (int)((3 * P.psb + (int64_t)P.K * P.ldb) * 4), 0x00020000);
  int offa[C::NA], offb[C::NB][2];
#pragma unroll
  for (int t = 0; t < C::NA; ++t) offa[t] = (int)(((int64_t)rowa[t] * P.lda + 4 * kqa) * 4);
#pragma unroll
  for (int t = 0; t < C::NB; ++t)
#pragma unroll
    for (int e = 0; e < 2; ++e) offb[t][e] = (int)(((int64_t)(2 * kb(t) + e) * P.ldb + colb) * 4);

  floatx4 acc[4][C::TM][C::TN];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) acc[p][i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  floatx4 ra[4][C::NA], rb[4][C::NB][2];

  // FAST: whole tile and whole K step (no clamping, no masking)
  auto load_a = [&](int k0, auto fast) __attribute__((always_inline)) {
    constexpr bool FAST = decltype(fast)::value;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < C::NA; ++t) {
        if constexpr (BUF && FAST) {
          ra[q][t] = buf_load4(srcA, offa[t], (int)((q * P.psa + k0) * 4));
        } else if constexpr (BUF) {
          ra[q][t] = buf_load4(srcA, offa[t] + 4 * (min(k0 + 4 * kqa, lastk) - 4 * kqa), (int)(q * P.psa * 4));
        } else {
          const float* Ar = P.A + q * P.psa + (int64_t)rowa[t] * P.lda;
#pragma unroll
          for (int e = 0; e < 4; ++e) ra[q][t][e] = gload(Ar, min(k0 + 4 * kqa + e, P.K - 1));
        }
      }
  };
  auto load_b = [&](int k0, auto fast) __attribute__((always_inline)) {
    constexpr bool FAST = decltype(fast)::value;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < C::NB; ++t)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int gk = min(k0 + 2 * kb(t) + e, P.K - 1);
          if constexpr (BUF && FAST) {
            rb[q][t][e] = buf_load4(srcB, offb[t][e], (int)((q * P.psb + (int64_t)k0 * P.ldb) * 4));
          } else if constexpr (BUF) {
            rb[q][t][e] = buf_load4(srcB, (int)(((int64_t)gk * P.ldb + colb) * 4), (int)(q * P.psb * 4));
          } else {
            const float* Bk = P.B + q * P.psb + (int64_t)gk * P.ldb;
#pragma unroll
            for (int c = 0; c < 4; ++c) rb[q][t][e][c] = gload(Bk, min(n0 + 4 * jqb + c, P.N - 1));
          }
        }
  };
  auto store_a = [&](__bf16* As, int k0, auto fast) __attribute__((always_inline)) {
    constexpr bool FAST = decltype(fast)::value;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < C::NA; ++t) {
        const int i = (tid + t * C::NT) / 8;
        floatx4 v = ra[q][t];
        if constexpr (!FAST) {
          const bool rok = m0 + i < P.M;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (rok && k0 + 4 * kqa + e < P.K) ? v[e] : 0.f;
        }
        *reinterpret_cast<bf16x4*>(&As[db_off(q * BM + i, kqa >> 1) + (kqa & 1) * 4]) =
            __builtin_convertvector(v, bf16x4);
      }
  };
  auto store_b = [&](__bf16* As, int k0, auto fast) __attribute__((always_inline)) {
    constexpr bool FAST = decltype(fast)::value;
    __bf16* const Bs = As + 4 * BM * BK;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < C::NB; ++t) {
        const int kk = 2 * kb(t);  // k within the step, even
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          floatx2 v = {rb[q][t][0][c], rb[q][t][1][c]};
          if constexpr (!FAST) {
            const bool cok = n0 + 4 * jqb + c < P.N;
            v[0] = (cok && k0 + kk < P.K) ? v[0] : 0.f;
            v[1] = (cok && k0 + kk + 1 < P.K) ? v[1] : 0.f;
          }
          *reinterpret_cast<bf16x2*>(&Bs[db_off(q * BN + 4 * jqb + c, kk >> 3) + (kk & 7)]) =
              __builtin_convertvector(v, bf16x2);
        }
      }
  };

  const int fr = lane & 15, fc = lane >> 4;
  bf16x8 b[C::TN][4];
  auto frag_b = [&](const __bf16* As) __attribute__((always_inline)) {
    const __bf16* const Bs = As + 4 * BM * BK;
#pragma unroll
    for (int j = 0; j < C::TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        b[j][q] = *reinterpret_cast<const bf16x8*>(&Bs[db_off(q * BN + wn * C::WTN + j * 16 + fr, fc)]);
  };
  // MFMAs of wave-tile rows i0 <= i < i1 (compile-time bounds after inlining)
  auto compute = [&](const __bf16* As, int i0, int i1) __attribute__((always_inline)) {
#pragma unroll
    for (int i = i0; i < i1; ++i) {
      bf16x8 a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        a[q] = *reinterpret_cast<const bf16x8*>(&As[db_off(q * BM + wm * C::WTM + i * 16 + fr, fc)]);
      const bf16x8 na1 = neg_bf16x8(a[1]), na2 = neg_bf16x8(a[2]), na3 = neg_bf16x8(a[3]);
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        // Hamilton product: acc_p += sum_q sign(p, q) a_q b_{r(p, q)}, the four planes interleaved
        acc[0][i][j] = mma_bf16(a[0], b[j][0], acc[0][i][j]);
        acc[1][i][j] = mma_bf16(a[0], b[j][1], acc[1][i][j]);
        acc[2][i][j] = mma_bf16(a[0], b[j][2], acc[2][i][j]);
        acc[3][i][j] = mma_bf16(a[0], b[j][3], acc[3][i][j]);
        acc[0][i][j] = mma_bf16(na1, b[j][1], acc[0][i][j]);
        acc[1][i][j] = mma_bf16(a[1], b[j][0], acc[1][i][j]);
        acc[2][i][j] = mma_bf16(na1, b[j][3], acc[2][i][j]);
        acc[3][i][j] = mma_bf16(a[1], b[j][2], acc[3][i][j]);
        acc[0][i][j] = mma_bf16(na2, b[j][2], acc[0][i][j]);
        acc[1][i][j] = mma_bf16(a[2], b[j][3], acc[1][i][j]);
        acc[2][i][j] = mma_bf16(a[2], b[j][0], acc[2][i][j]);
        acc[3][i][j] = mma_bf16(na2, b[j][1], acc[3][i][j]);
        acc[0][i][j] = mma_bf16(na3, b[j][3], acc[0][i][j]);
        acc[1][i][j] = mma_bf16(na3, b[j][2], acc[1][i][j]);
        acc[2][i][j] = mma_bf16(a[3], b[j][1], acc[2][i][j]);
        acc[3][i][j] = mma_bf16(a[3], b[j][0], acc[3][i][j]);
      }
    }
  };

  constexpr int IH = C::TM / 2;
  // The whole K loop, fast (whole tile, K a multiple of the step: no clamping, no masking) or not.
  // The last step is peeled so that every loop step stages the next tile unconditionally.
  auto run = [&](auto fast) __attribute__((always_inline)) {
    const int nk = (P.K + BK - 1) / BK;
    load_a(0, fast);
    load_b(0, fast);
    store_a(smem, 0, fast);
    store_b(smem, 0, fast);
    __syncthreads();
    for (int kt = 0; kt + 1 < nk; ++kt) {
      __bf16* const cur = smem + (kt & 1) * C::STAGE;
      __bf16* const nxt = smem + ((kt + 1) & 1) * C::STAGE;
      const int kn = (kt + 1) * BK;
      frag_b(cur);
      load_a(kn, fast);
      compute(cur, 0, IH);
      store_a(nxt, kn, fast);
      load_b(kn, fast);
      compute(cur, IH, C::TM);
      store_b(nxt, kn, fast);
      __syncthreads();
    }
    const __bf16* const last = smem + ((nk - 1) & 1) * C::STAGE;
    frag_b(last);
    compute(last, 0, C::TM);
    __syncthreads();  // the next tile's first stage overwrites LDS
  };
  if (P.K > 0) {
    if (full_mn && P.K % BK == 0)
      run(std::integral_constant<bool, true>{});
    else
      run(std::integral_constant<bool, false>{});
  }

#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int rb0 = m0 + wm * C::WTM + i * 16 + 4 * fc, cb0 = n0 + wn * C::WTN + j * 16 + fr;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        float inv[4][3];
#pragma unroll
        for (int r = 0; r < 4; ++r) epilogue_inputs(P, p, rb0 + r, cb0, inv[r]);
#pragma unroll
        for (int r = 0; r < 4; ++r) epilogue_apply(P, p, rb0 + r, cb0, acc[p][i][j][r], inv[r], s_d, s_x);
      }
    }
}

template <int BM, int BN, int WM, int WN, bool BUF, int MINW>
__global__ void __launch_bounds__(64 * WM * WN, MINW) qgemm_bf16_db_kernel(GemmParams<float> P) {
  using C = Bf16DbCfg<BM, BN, WM, WN>;
  __shared__ __attribute__((aligned(16))) __bf16 smem[2 * C::STAGE];
  __shared__ double red_lds[C::NW][2];
  const int nt = P.tiles_m * P.tiles_n;
  double s_d = 0.0, s_x = 0.0;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int tm, tn;
    tile_of_block(t, nt, P.tiles_m, P.tiles_n, tm, tn);
    bf16_db_tile<BM, BN, WM, WN, BUF>(P, tm, tn, smem, s_d, s_x);
  }
  store_partials<C::NW>(P.partial, s_d, s_x, red_lds, threadIdx.x & 63, threadIdx.x >> 6, threadIdx.x);
}

// Buffer loads need 16-byte aligned bases, leading dimensions and plane strides (P.vec) and byte
// offsets below 2^31 over the four planes.
static bool bf16_buffer_ok(const GemmParams<float>& P) {
  const int64_t lim = int64_t(1) << 31;
  return P.vec && (3 * P.psa + (int64_t)P.M * P.lda) * 4 < lim && (3 * P.psb + (int64_t)P.K * P.ldb) * 4 < lim;
}

template <int BM, int BN, int WM, int WN, int MINW>
static int64_t launch_bf16_db(const GemmParams<float>& P0, int per_cu, hipStream_t s) {
  using C = Bf16DbCfg<BM, BN, WM, WN>;
  GemmParams<float> P = P0;
  P.tiles_m = (P.M + BM - 1) / BM;
  P.tiles_n = (P.N + BN - 1) / BN;
  const int64_t nt = (int64_t)P.tiles_m * P.tiles_n;
  if (nt == 0) return 0;
  auto kern = bf16_buffer_ok(P) ? qgemm_bf16_db_kernel<BM, BN, WM, WN, true, MINW>
                                : qgemm_bf16_db_kernel<BM, BN, WM, WN, false, MINW>;
  LaunchShape ls;
  ls.grid = nt;
  if (per_cu > 0) {
    static const std::pair<int, size_t> kl = [&] {
      int occ = 0;
      QP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, C::NT, 0));
      hipFuncAttributes fa{};
      QP_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)));
      return std::make_pair(std::max(occ, 1), (size_t)fa.sharedSizeBytes);
    }();
    ls = launch_shape(nt, per_cu, kl.first, kl.second);
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)ls.grid), dim3(C::NT), ls.dyn_lds, s, P);
  QP_HIP(hipGetLastError());
  return ls.grid;
}

template <int BM, int BN, int WM, int WN>
static int64_t launch_bf16(const GemmParams<float>& P0, int per_cu, hipStream_t s) {
  using C = Bf16Cfg<BM, BN, WM, WN>;
  GemmParams<float> P = P0;
  P.tiles_m = (P.M + BM - 1) / BM;
  P.tiles_n = (P.N + BN - 1) / BN;
  const int64_t nt = (int64_t)P.tiles_m * P.tiles_n;
  if (nt == 0) return 0;
  auto kern = qgemm_bf16_kernel<BM, BN, WM, WN>;
  LaunchShape ls;
  ls.grid = nt;
  if (per_cu > 0) {
    static const std::pair<int, size_t> kl = [&] {
      int occ = 0;
      QP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, C::NT, 0));
      hipFuncAttributes fa{};
      QP_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)));
      return std::make_pair(std::max(occ, 1), (size_t)fa.sharedSizeBytes);
    }();
    ls = launch_shape(nt, per_cu, kl.first, kl.second);
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)ls.grid), dim3(C::NT), ls.dyn_lds, s, P);
  QP_HIP(hipGetLastError());
  return ls.grid;
}

// ---------------------------------------------------------------------------------------------------
// Staged form: the product first writes BF16 copies of its operands into the context's stage buffer,
// A as [plane][Mp][Kp] and B transposed as [plane][Np][Kp] (both k-contiguous, rows of Kp = K rounded
// up to 32, Mp and Np rounded up to the tile, zeros in the padding), then runs a kernel that reads
// only those copies: no masks, no clamps, no conversion or transposition in the K loop, and half the
// staging registers of the FP32-operand form, which leaves room for larger tiles.  The copies are
// rounded to nearest even exactly as the other forms round while staging, and the MFMA sequence over
// k is the same, so the three forms give identical products.
// BF16 MFMA shapes of the staged form.  Fragments are 8 consecutive k of one row (A) or column (B) per
// lane, i.e. one 16-byte LDS chunk; chunk(l, h) names the chunk (of the 4 in a 32-k row) that lane l
// reads for k sub-step h.  Output register r of lane l holds element (crow(l, r), ccol(l)) of the block.
struct BfM16 {  // v_mfma_f32_16x16x32_bf16: one 32-k sub-step per K step
  using Acc = floatx4;
  static constexpr int BLK = 16, KSUB = 1, NR = 4;
  __device__ static int fr(int l) { return l & 15; }
  __device__ static int chunk(int l, int) { return l >> 4; }
  __device__ static int crow(int l, int r) { return ((l >> 4) << 2) + r; }
  __device__ static int ccol(int l) { return l & 15; }
  __device__ static Acc mma(bf16x8 a, bf16x8 b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
struct BfM32 {  // v_mfma_f32_32x32x16_bf16: two 16-k sub-steps per K step
  using Acc = floatx16;
  static constexpr int BLK = 32, KSUB = 2, NR = 16;
  __device__ static int fr(int l) { return l & 31; }
  __device__ static int chunk(int l, int h) { return 2 * h + (l >> 5); }
  __device__ static int crow(int l, int r) { return ((r >> 2) << 3) + ((l >> 5) << 2) + (r & 3); }
  __device__ static int ccol(int l) { return l & 31; }
  __device__ static Acc mma(bf16x8 a, bf16x8 b, Acc c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};

template <int BM, int BN, int WM, int WN, class MB = BfM16>
struct Bf16SCfg {
  static constexpr int BK = 32;
  static constexpr int NW = WM * WN, NT = 64 * NW;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / MB::BLK, TN = WTN / MB::BLK;
  static constexpr int ITEMS = TM * MB::KSUB;  // (row block, k sub-step) pairs of one K step
  static constexpr int ACH = BM * 4, BCH = BN * 4;  // 16-byte chunks (8 k) of one plane tile
  static constexpr int NA = (ACH + NT - 1) / NT, NB = (BCH + NT - 1) / NT;
  static constexpr int STAGE = 4 * (BM + BN) * BK;  // bf16 elements of one LDS stage
  static_assert(ITEMS >= 2 && TN >= 1 && WTM % MB::BLK == 0 && WTN % MB::BLK == 0, "wave tile (two halves)");
  static_assert(2 * STAGE * 2 <= 160 * 1024, "two stages fit the LDS");
};

// The BF16 copies of one product: planes of rows x kp elements (kp a multiple of 32).
struct Bf16Stage {
  const __bf16* a;  // [4][mp][kp]
  const __bf16* b;  // [4][np][kp] (B transposed)
  int mp, np, kp;
};

// DIRECT: the operand tiles go from the stage buffer straight to LDS (16-byte buffer loads with an LDS
// destination) instead of through registers, which frees the staging registers for larger tiles.
template <int BM, int BN, int WM, int WN, class MB, bool PRIO = false, bool DIRECT = false>
__device__ __forceinline__ void bf16s_tile(const GemmParams<float>& P, const Bf16Stage& S, int tm, int tn,
                                           __bf16* smem, double& s_d, double& s_x) {
  using C = Bf16SCfg<BM, BN, WM, WN, MB>;
  using Acc = typename MB::Acc;
  constexpr int BK = C::BK;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w % WM, wn = w / WM;
  // raw buffers over the four planes of each copy (extents below 2^31 bytes, checked by the launcher)
  const __amdgpu_buffer_rsrc_t srcA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<__bf16*>(S.a), (short)0, (int)((int64_t)4 * S.mp * S.kp * 2), 0x00020000);
  const __amdgpu_buffer_rsrc_t srcB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<__bf16*>(S.b), (short)0, (int)((int64_t)4 * S.np * S.kp * 2), 0x00020000);
  const int psa = S.mp * S.kp * 2, psb = S.np * S.kp * 2;  // plane strides in bytes
  // chunk c = tid + t NT of a plane tile: row c / 4, k 8 (c % 4) .. +7
  int offa[C::NA], offb[C::NB];
#pragma unroll
  for (int t = 0; t < C::NA; ++t) {
    const int c = min(tid + t * C::NT, C::ACH - 1);
    offa[t] = ((m0 + c / 4) * S.kp + 8 * (c % 4)) * 2;
  }
#pragma unroll
  for (int t = 0; t < C::NB; ++t) {
    const int c = min(tid + t * C::NT, C::BCH - 1);
    offb[t] = ((n0 + c / 4) * S.kp + 8 * (c % 4)) * 2;
  }

  Acc acc[4][C::TM][C::TN];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) acc[p][i][j] = Acc{};

  u32x4 ra[4][C::NA], rb[4][C::NB];
  auto load_a = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < C::NA; ++t)
        ra[q][t] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(srcA, offa[t], q * psa + 2 * k0, 0));
  };
  auto load_b = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < C::NB; ++t)
        rb[q][t] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(srcB, offb[t], q * psb + 2 * k0, 0));
  };
  auto store_a = [&](__bf16* As) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < C::NA; ++t) {
        const int c = tid + t * C::NT;
        if (C::ACH % C::NT == 0 || c < C::ACH) *reinterpret_cast<u32x4*>(&As[db_off(q * BM + c / 4, c % 4)]) = ra[q][t];
      }
  };
  auto store_b = [&](__bf16* As) __attribute__((always_inline)) {
    __bf16* const Bs = As + 4 * BM * BK;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < C::NB; ++t) {
        const int c = tid + t * C::NT;
        if (C::BCH % C::NT == 0 || c < C::BCH) *reinterpret_cast<u32x4*>(&Bs[db_off(q * BN + c / 4, c % 4)]) = rb[q][t];
      }
  };

  const int fr = MB::fr(lane);
  bf16x8 b[C::TN][MB::KSUB][4];
  auto frag_b = [&](const __bf16* As) __attribute__((always_inline)) {
    const __bf16* const Bs = As + 4 * BM * BK;
#pragma unroll
    for (int j = 0; j < C::TN; ++j)
#pragma unroll
      for (int h = 0; h < MB::KSUB; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          b[j][h][q] = *reinterpret_cast<const bf16x8*>(
              &Bs[db_off(q * BN + wn * C::WTN + j * MB::BLK + fr, MB::chunk(lane, h))]);
  };
  // MFMAs of the (row block, k sub-step) items it0 <= it < it1 (compile-time bounds after inlining)
  auto compute = [&](const __bf16* As, int it0, int it1) __attribute__((always_inline)) {
    // PRIO: the wave's issue priority is raised while it has MFMAs to issue, so that the LDS and global
    // traffic of the other waves fills the gaps instead of delaying them
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int it = it0; it < it1; ++it) {
      const int i = it / MB::KSUB, h = it % MB::KSUB;
      bf16x8 a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        a[q] = *reinterpret_cast<const bf16x8*>(&As[db_off(q * BM + wm * C::WTM + i * MB::BLK + fr, MB::chunk(lane, h))]);
      const bf16x8 na1 = neg_bf16x8(a[1]), na2 = neg_bf16x8(a[2]), na3 = neg_bf16x8(a[3]);
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const bf16x8(&bb)[4] = b[j][h];
        acc[0][i][j] = MB::mma(a[0], bb[0], acc[0][i][j]);
        acc[1][i][j] = MB::mma(a[0], bb[1], acc[1][i][j]);
        acc[2][i][j] = MB::mma(a[0], bb[2], acc[2][i][j]);
        acc[3][i][j] = MB::mma(a[0], bb[3], acc[3][i][j]);
        acc[0][i][j] = MB::mma(na1, bb[1], acc[0][i][j]);
        acc[1][i][j] = MB::mma(a[1], bb[0], acc[1][i][j]);
        acc[2][i][j] = MB::mma(na1, bb[3], acc[2][i][j]);
        acc[3][i][j] = MB::mma(a[1], bb[2], acc[3][i][j]);
        acc[0][i][j] = MB::mma(na2, bb[2], acc[0][i][j]);
        acc[1][i][j] = MB::mma(a[2], bb[3], acc[1][i][j]);
        acc[2][i][j] = MB::mma(a[2], bb[0], acc[2][i][j]);
        acc[3][i][j] = MB::mma(na2, bb[1], acc[3][i][j]);
        acc[0][i][j] = MB::mma(na3, bb[3], acc[0][i][j]);
        acc[1][i][j] = MB::mma(na3, bb[2], acc[1][i][j]);
        acc[2][i][j] = MB::mma(a[3], bb[1], acc[2][i][j]);
        acc[3][i][j] = MB::mma(a[3], bb[0], acc[3][i][j]);
      }
    }
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
  };

  constexpr int IH = C::ITEMS / 2;
  const int nk = S.kp / BK;
  if constexpr (DIRECT) {
    // One instruction per wave fills 16 LDS rows (64 bytes each) of one plane, lane l at byte 16 l: row
    // 16 blk + l / 4, slot l % 4, which db_off gives the chunk (l % 4) ^ ((row >> 1) & 3) of that row.
    constexpr int NIA = 4 * BM / 16, NI = NIA + 4 * BN / 16;
    static_assert(NI % C::NW == 0, "whole LDS-direct instructions per wave");
    auto issue = [&](__bf16* St, int k0) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < NI / C::NW; ++u) {
        const int i = w + u * C::NW;  // wave-uniform
        const bool isA = i < NIA;
        const int ii = isA ? i : i - NIA;
        const int rows = isA ? BM : BN;
        const int q = ii / (rows / 16), blk = ii % (rows / 16);
        const int row = 16 * blk + (lane >> 2);
        const int c = (lane & 3) ^ ((row >> 1) & 3);
        const int voff = (((isA ? m0 : n0) + row) * S.kp + 8 * c) * 2;
        const int soff = q * (isA ? psa : psb) + 2 * k0;
        __bf16* const dst = St + (isA ? 0 : 4 * BM * BK) + (q * rows + 16 * blk) * BK;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(isA ? srcA : srcB, (__attribute__((address_space(3))) void*)dst, 16,
                                                 voff, soff, 0, 0);
      }
    };
    if (nk > 0) {
      __syncthreads();  // the caller may have used the LDS just before (previous tile)
      issue(smem, 0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      for (int kt = 0; kt < nk; ++kt) {
        __bf16* const cur = smem + (kt & 1) * C::STAGE;
        // the other stage was last read in step kt - 1, before the barrier that ended it
        if (kt + 1 < nk) issue(smem + ((kt + 1) & 1) * C::STAGE, (kt + 1) * BK);
        if constexpr (C::TM == 1 && MB::KSUB > 1) {
          // one row block per wave: the B fragments of one k sub-step at a time (half the registers; the
          // same LDS reads and the same MFMA sequence)
#pragma unroll
          for (int h = 0; h < MB::KSUB; ++h) {
            const __bf16* const Bs = cur + 4 * BM * BK;
#pragma unroll
            for (int j = 0; j < C::TN; ++j)
#pragma unroll
              for (int q = 0; q < 4; ++q)
                b[j][h][q] = *reinterpret_cast<const bf16x8*>(
                    &Bs[db_off(q * BN + wn * C::WTN + j * MB::BLK + fr, MB::chunk(lane, h))]);
            compute(cur, h, h + 1);
          }
        } else {
          frag_b(cur);
          compute(cur, 0, C::ITEMS);
        }
        __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of step kt + 1 are in LDS
        __syncthreads();
      }
    }
  } else if (nk > 0) {
    load_a(0);
    load_b(0);
    store_a(smem);
    store_b(smem);
    __syncthreads();
    for (int kt = 0; kt + 1 < nk; ++kt) {
      __bf16* const cur = smem + (kt & 1) * C::STAGE;
      __bf16* const nxt = smem + ((kt + 1) & 1) * C::STAGE;
      const int kn = (kt + 1) * BK;
      frag_b(cur);
      load_a(kn);
      compute(cur, 0, IH);
      store_a(nxt);
      load_b(kn);
      compute(cur, IH, C::ITEMS);
      store_b(nxt);
      __syncthreads();
    }
    const __bf16* const last = smem + ((nk - 1) & 1) * C::STAGE;
    frag_b(last);
    compute(last, 0, C::ITEMS);
    __syncthreads();  // the next tile's first stage overwrites LDS
  }

#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int rb = m0 + wm * C::WTM + i * MB::BLK, cb = n0 + wn * C::WTN + j * MB::BLK + MB::ccol(lane);
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int r0 = 0; r0 < MB::NR; r0 += 4) {  // inputs of 4 elements in flight at a time
          float inv[4][3];
#pragma unroll
          for (int r = 0; r < 4; ++r) epilogue_inputs(P, p, rb + MB::crow(lane, r0 + r), cb, inv[r]);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            epilogue_apply(P, p, rb + MB::crow(lane, r0 + r), cb, acc[p][i][j][r0 + r], inv[r], s_d, s_x);
        }
    }
}

template <int BM, int BN, int WM, int WN, int MINW, class MB, bool PRIO, bool DIRECT>
__global__ void __launch_bounds__(64 * WM * WN, MINW) qgemm_bf16s_kernel(GemmParams<float> P, Bf16Stage S) {
  using C = Bf16SCfg<BM, BN, WM, WN, MB>;
  __shared__ __attribute__((aligned(16))) __bf16 smem[2 * C::STAGE];
  __shared__ double red_lds[C::NW][2];
  const int nt = P.tiles_m * P.tiles_n;
  double s_d = 0.0, s_x = 0.0;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int tm, tn;
    tile_of_block(t, nt, P.tiles_m, P.tiles_n, tm, tn);
    bf16s_tile<BM, BN, WM, WN, MB, PRIO, DIRECT>(P, S, tm, tn, smem, s_d, s_x);
  }
  store_partials<C::NW>(P.partial, s_d, s_x, red_lds, threadIdx.x & 63, threadIdx.x >> 6, threadIdx.x);
}

// Split operands (three-product form): x = hi + lo + d with hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in
// FP32) and |d| <= 2^-16 |x|.  Rows of the split copies hold 3 kp elements, three segments of kp along k:
// A as [hi | hi | lo] and B (transposed) as [hi | lo | hi], so that one product over 3 kp sums
// hi.hi + hi.lo + lo.hi; the dropped lo.lo term and d bound the error by about 3 2^-16 |a||b| per term.
enum : int { kSplitNone = 0, kSplitA = 1, kSplitB = 2 };

// Eight consecutive k of one row (x0: the first four, x1: the next four) to the copy at column k of `row`.
__device__ __forceinline__ void split_store(__bf16* __restrict__ row, int kp, int k, const floatx4& x0,
                                            const floatx4& x1, int split) {
  bf16x8 h, l;
  const bf16x4 h0 = __builtin_convertvector(x0, bf16x4), h1 = __builtin_convertvector(x1, bf16x4);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    h[e] = h0[e];
    h[e + 4] = h1[e];
  }
  *reinterpret_cast<bf16x8*>(row + k) = h;
  if (split == kSplitNone) return;
  floatx4 r0, r1;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    r0[e] = x0[e] - (float)h0[e];
    r1[e] = x1[e] - (float)h1[e];
  }
  const bf16x4 l0 = __builtin_convertvector(r0, bf16x4), l1 = __builtin_convertvector(r1, bf16x4);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    l[e] = l0[e];
    l[e + 4] = l1[e];
  }
  *reinterpret_cast<bf16x8*>(row + kp + k) = split == kSplitA ? h : l;
  *reinterpret_cast<bf16x8*>(row + 2 * kp + k) = split == kSplitA ? l : h;
}

// out[q][r][8c .. 8c+7] = bf16(A[q][r][8c ..]) inside the matrix, 0 in the padding (r < mp, 8c < kp); rows
// of kp elements, or of 3 kp for split copies.  vec: 16-byte aligned base, lda and psa.
__global__ void __launch_bounds__(256) bf16_rows_kernel(const float* __restrict__ A, int64_t lda, int64_t psa, int M,
                                                        int K, __bf16* __restrict__ out, int mp, int kp, int vec,
                                                        int split) {
  const int64_t chunks = (int64_t)4 * mp * (kp / 8);
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < chunks; c += (int64_t)gridDim.x * blockDim.x) {
    const int kc = (int)(c % (kp / 8));
    const int64_t qr = c / (kp / 8);
    const int r = (int)(qr % mp), q = (int)(qr / mp);
    floatx4 lo = {0.f, 0.f, 0.f, 0.f}, hi = {0.f, 0.f, 0.f, 0.f};
    if (r < M) {
      const float* row = A + q * psa + (int64_t)r * lda;
      if (vec && 8 * kc + 8 <= K) {  // whole chunk: two 16-byte loads
        lo = gload(reinterpret_cast<const floatx4*>(row + 8 * kc), 0);
        hi = gload(reinterpret_cast<const floatx4*>(row + 8 * kc + 4), 0);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = 8 * kc + e;
          lo[e] = k < K ? gload(row, k) : 0.f;
          hi[e] = k + 4 < K ? gload(row, k + 4) : 0.f;
        }
      }
    }
    const int64_t rl = split == kSplitNone ? kp : 3 * (int64_t)kp;
    split_store(out + qr * rl, kp, 8 * kc, lo, hi, split);
  }
}

// out[q][n][k] = bf16(B[q][k][n]) inside the matrix, 0 in the padding (n < np, k < kp): one 32 (k) x 64 (n)
// tile per workgroup through LDS, reads along n (16 bytes a lane when vec: 16-byte aligned base, ldb and
// psb), writes 16 bytes (8 k) per lane; rows of kp elements, or of 3 kp for split copies.
__global__ void __launch_bounds__(256) bf16_transpose_kernel(const float* __restrict__ B, int64_t ldb, int64_t psb,
                                                             int K, int N, __bf16* __restrict__ out, int np, int kp,
                                                             int vec, int split) {
  __shared__ float tile[32][65];
  const int tk = kp / 32, tn = np / 64;
  const int64_t t = blockIdx.x;
  const int q = (int)(t / ((int64_t)tk * tn));
  const int rest = (int)(t % ((int64_t)tk * tn));
  const int k0 = (rest / tn) * 32, n0 = (rest % tn) * 64;
  const int tid = threadIdx.x;
  {
    // thread: columns n0 + 4 c .. +3 of rows k0 + r and k0 + r + 16
    const int c = tid % 16, r = tid / 16, n = n0 + 4 * c;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kr = r + 16 * h, k = k0 + kr;
      floatx4 v = {0.f, 0.f, 0.f, 0.f};
      if (k < K) {
        const float* row = B + q * psb + (int64_t)k * ldb;
        if (vec && n + 4 <= N) {
          v = gload(reinterpret_cast<const floatx4*>(row + n), 0);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = n + e < N ? gload(row, n + e) : 0.f;
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) tile[kr][4 * c + e] = v[e];
    }
  }
  __syncthreads();
  const int nl = tid / 4, kc = (tid % 4) * 8;
  floatx4 lo, hi;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    lo[e] = tile[kc + e][nl];
    hi[e] = tile[kc + 4 + e][nl];
  }
  const int64_t rl = split == kSplitNone ? kp : 3 * (int64_t)kp;
  split_store(out + ((int64_t)q * np + n0 + nl) * rl, kp, k0 + kc, lo, hi, split);
}

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Stage bytes of a staged product (rows padded to 128 cover every staged tile shape; split copies hold
// three segments per row).
static int64_t stage_bytes(int64_t M, int64_t N, int64_t K, bool split = false) {
  return (split ? 3 : 1) * 2 * 4 * (round_up(M, 128) + round_up(N, 128)) * round_up(std::max<int64_t>(K, 1), 32);
}

// The split copies' buffer loads take byte offsets below 2^31 over the four planes.
bool bf16x3_fits(int64_t M, int64_t N, int64_t K) {
  return 4 * std::max(round_up(M, 128), round_up(N, 128)) * 3 * std::max<int64_t>(round_up(K, 32), 32) * 2 <
         (int64_t(1) << 31);
}

// SPLIT: the three-product form (operands split into BF16 hi and lo, products summed over 3 kp).
// DIRECT: operand tiles loaded straight into LDS.
template <int BM, int BN, int WM, int WN, int MINW, class MB = BfM16, bool PRIO = false, bool SPLIT = false,
          bool DIRECT = false>
static int64_t launch_bf16_staged(const GemmParams<float>& P0, int per_cu, hipStream_t s, GemmScratch& sc) {
  using C = Bf16SCfg<BM, BN, WM, WN, MB>;
  GemmParams<float> P = P0;
  P.tiles_m = (P.M + BM - 1) / BM;
  P.tiles_n = (P.N + BN - 1) / BN;
  const int64_t nt = (int64_t)P.tiles_m * P.tiles_n;
  if (nt == 0) return 0;
  const int64_t mp = round_up(P.M, 128), np = round_up(P.N, 128), kp = round_up(P.K, 32);
  // copies beyond the 32-bit offsets of the buffer loads (about 16k x 16k): the direct form, which rounds
  // while staging and takes any size, computes the same products (the split form has no direct form)
  if (SPLIT && !bf16x3_fits(P.M, P.N, P.K))
    throw Error(-1, "qgemm: the split BF16 product's copies exceed 2^31 bytes");
  if (!SPLIT && 4 * std::max(mp, np) * std::max<int64_t>(kp, 32) * 2 >= (int64_t(1) << 31))
    return launch_bf16_db<64, 64, 2, 2, 2>(P0, 0, s);
  const int64_t kps = SPLIT ? 3 * kp : kp;  // staged row length
  const size_t need = (size_t)stage_bytes(P.M, P.N, P.K, SPLIT);
  if (sc.stage_bytes < need) {
    if (sc.no_grow)
      throw Error(-1, "qgemm: the staged BF16 product needs a " + std::to_string(need) +
                          "-byte stage buffer, which an allocation-free call cannot grow");
    // grow the stage buffer (kernels of earlier products on the stream may still read it)
    QP_HIP(hipStreamSynchronize(s));
    if (sc.stage) QP_HIP(hipFree(sc.stage));
    sc.stage = nullptr;
    sc.stage_bytes = 0;
    if (hipMalloc(&sc.stage, need) != hipSuccess || !sc.stage) {
      (void)hipGetLastError();
      sc.stage = nullptr;
      throw Error(-6, "qgemm: allocation of the BF16 stage buffer (" + std::to_string(need) + " bytes) failed");
    }
    sc.stage_bytes = need;
  }
  __bf16* const a16 = static_cast<__bf16*>(sc.stage);
  __bf16* const b16 = a16 + 4 * mp * kps;
  if (kp > 0) {
    const int64_t chunks = 4 * mp * (kp / 8);
    const int64_t grid_r = std::min<int64_t>((chunks + 255) / 256, 65536);
    const int vec_a = (reinterpret_cast<uintptr_t>(P.A) & 15) == 0 && P.lda % 4 == 0 && P.psa % 4 == 0;
    hipLaunchKernelGGL(bf16_rows_kernel, dim3((unsigned)grid_r), dim3(256), 0, s, P.A, P.lda, P.psa, P.M, P.K, a16,
                       (int)mp, (int)kp, vec_a, SPLIT ? (int)kSplitA : (int)kSplitNone);
    QP_HIP(hipGetLastError());
    const int64_t grid_t = 4 * (kp / 32) * (np / 64);
    const int vec_b = (reinterpret_cast<uintptr_t>(P.B) & 15) == 0 && P.ldb % 4 == 0 && P.psb % 4 == 0;
    hipLaunchKernelGGL(bf16_transpose_kernel, dim3((unsigned)grid_t), dim3(256), 0, s, P.B, P.ldb, P.psb, P.K, P.N, b16,
                       (int)np, (int)kp, vec_b, SPLIT ? (int)kSplitB : (int)kSplitNone);
    QP_HIP(hipGetLastError());
  }
  const Bf16Stage S{a16, b16, (int)mp, (int)np, (int)kps};
  auto kern = qgemm_bf16s_kernel<BM, BN, WM, WN, MINW, MB, PRIO, DIRECT>;
  LaunchShape ls;
  ls.grid = nt;
  if (per_cu > 0) {
    static const std::pair<int, size_t> kl = [&] {
      int occ = 0;
      QP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, C::NT, 0));
      hipFuncAttributes fa{};
      QP_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)));
      return std::make_pair(std::max(occ, 1), (size_t)fa.sharedSizeBytes);
    }();
    ls = launch_shape(nt, per_cu, kl.first, kl.second);
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)ls.grid), dim3(C::NT), ls.dyn_lds, s, P, S);
  QP_HIP(hipGetLastError());
  return ls.grid;
}

struct Bf16Entry {
  TileConfig cfg;
  int64_t (*fn)(const GemmParams<float>&, int, hipStream_t, GemmScratch&);
};

// The forms that read the FP32 operands directly leave the stage buffer alone.
template <int64_t (*F)(const GemmParams<float>&, int, hipStream_t)>
static int64_t direct(const GemmParams<float>& P, int per_cu, hipStream_t s, GemmScratch&) {
  return F(P, per_cu, s);
}

static const std::vector<Bf16Entry>& bf16_table() {
  static const std::vector<Bf16Entry> t = {
      // Measured on MI355X at 4096^3 (2048^3): 8 reaches 1060 (910) TFLOP/s including its operand copies,
      // 6 960-1000 (900-920), 0 790 (850), 5 (the single-buffered form) 490; below about 4 tiles of
      // 64 x 64 per compute unit the copies cost more than they save, and below 1 the 32 x 32 tiles win.
      // Tiles of 128 x 128 (staged) measured 320-360 TFLOP/s: their LDS stages leave one workgroup per CU.
      // 9 and 10 (32 x 32 x 16 MFMA, sums rounded in another order) measured 1020 and 1080, within the
      // run-to-run spread of 8, whose products equal those of the direct forms bit for bit.  8 raises
      // its waves' issue priority around the MFMA blocks: 2-3% faster in the same run at 2048^3 and 4096^3.
      {{0, 64, 64, 32, 256, "bf16_64x64x32_w2x2_mfma16x16x32_db_occ2"}, direct<launch_bf16_db<64, 64, 2, 2, 2>>},
      {{1, 32, 32, 32, 256, "bf16_32x32x32_w2x2_mfma16x16x32"}, direct<launch_bf16<32, 32, 2, 2>>},
      {{2, 64, 64, 32, 256, "bf16_64x64x32_w2x2_mfma16x16x32_db_occ2_cu2", 2}, direct<launch_bf16_db<64, 64, 2, 2, 2>>},
      {{3, 32, 32, 32, 256, "bf16_32x32x32_w2x2_mfma16x16x32_cu3", 3}, direct<launch_bf16<32, 32, 2, 2>>},
      {{4, 64, 128, 32, 512, "bf16_64x128x32_w2x4_mfma16x16x32_db"}, direct<launch_bf16_db<64, 128, 2, 4, 2>>},
      {{5, 64, 64, 32, 256, "bf16_64x64x32_w2x2_mfma16x16x32"}, direct<launch_bf16<64, 64, 2, 2>>},
      {{6, 64, 64, 32, 256, "bf16_64x64x32_w2x2_mfma16x16x32_staged"}, launch_bf16_staged<64, 64, 2, 2, 2>},
      {{7, 64, 64, 32, 256, "bf16_64x64x32_w2x2_mfma16x16x32_staged_cu2", 2}, launch_bf16_staged<64, 64, 2, 2, 2>},
      {{8, 64, 64, 32, 512, "bf16_64x64x32_w2x4_mfma16x16x32_staged"}, launch_bf16_staged<64, 64, 2, 4, 4, BfM16, true>},
      {{9, 64, 64, 32, 256, "bf16_64x64x32_w2x2_mfma32x32x16_staged"}, launch_bf16_staged<64, 64, 2, 2, 2, BfM32>},
      {{10, 128, 64, 32, 512, "bf16_128x64x32_w4x2_mfma32x32x16_staged"}, launch_bf16_staged<128, 64, 4, 2, 2, BfM32>},
      // Operand tiles loaded straight into LDS (no staging registers).  Measured at 4096^3 with the copies:
      // 11 1108-1127 TFLOP/s (the default above 1024 tiles of 64 x 64; its products equal 8's and the direct
      // forms' bit for bit), 12 (128 x 128, 16 waves of 32 x 32, one workgroup per CU) 1128-1168.  Dropped:
      // 128 x 64 with 8 waves (933-965), 128 x 128 with 8 waves of 64 x 32 (333: one workgroup of 8 waves
      // per CU), 128 x 128 with 16 waves on the 16 x 16 x 32 MFMA (634: spills in the K loop), 12 with the
      // issue priority raised around the MFMA blocks (1089; split 376 against 403).
      {{11, 64, 64, 32, 512, "bf16_64x64x32_w2x4_mfma16x16x32_staged_lds"},
       launch_bf16_staged<64, 64, 2, 4, 4, BfM16, true, false, true>},
      {{12, 128, 128, 32, 1024, "bf16_128x128x32_w4x4_mfma32x32x16_staged_lds"},
       launch_bf16_staged<128, 128, 4, 4, 4, BfM32, false, false, true>},
  };
  return t;
}

const std::vector<TileConfig>& bf16_configs() {
  static std::vector<TileConfig> v;
  if (v.empty())
    for (auto& e : bf16_table()) v.push_back(e.cfg);
  return v;
}

int64_t bf16_launch(const GemmParams<float>& P, int cfg, hipStream_t s, GemmScratch& scratch) {
  const auto& e = bf16_table().at(cfg);
  return e.fn(P, e.cfg.per_cu, s, scratch);
}

int64_t bf16_blocks(int cfg, int64_t M, int64_t N) {
  const auto& c = bf16_table().at(cfg).cfg;
  return ((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
}

// The three-product form: the staged kernels over the split copies.
static const std::vector<Bf16Entry>& bf16x3_table() {
  static const std::vector<Bf16Entry> t = {
      {{0, 64, 64, 32, 512, "bf16x3_64x64x32_w2x4_mfma16x16x32_staged"},
       launch_bf16_staged<64, 64, 2, 4, 4, BfM16, true, true>},
      {{1, 64, 64, 32, 256, "bf16x3_64x64x32_w2x2_mfma16x16x32_staged"},
       launch_bf16_staged<64, 64, 2, 2, 2, BfM16, false, true>},
      {{2, 128, 64, 32, 512, "bf16x3_128x64x32_w4x2_mfma32x32x16_staged"},
       launch_bf16_staged<128, 64, 4, 2, 2, BfM32, false, true>},
      // operand tiles straight into LDS; at 4096^3: 3 355-362 TFLOP/s of product flops (the default below 256
      // tiles of 128 x 128), 4 408-410 (the default from 256 such tiles), 0 342-345, 2 353-355
      {{3, 64, 64, 32, 512, "bf16x3_64x64x32_w2x4_mfma16x16x32_staged_lds"},
       launch_bf16_staged<64, 64, 2, 4, 4, BfM16, true, true, true>},
      {{4, 128, 128, 32, 1024, "bf16x3_128x128x32_w4x4_mfma32x32x16_staged_lds"},
       launch_bf16_staged<128, 128, 4, 4, 4, BfM32, false, true, true>},
  };
  return t;
}

const std::vector<TileConfig>& bf16x3_configs() {
  static std::vector<TileConfig> v;
  if (v.empty())
    for (auto& e : bf16x3_table()) v.push_back(e.cfg);
  return v;
}

int64_t bf16x3_launch(const GemmParams<float>& P, int cfg, hipStream_t s, GemmScratch& scratch) {
  const auto& e = bf16x3_table().at(cfg);
  return e.fn(P, e.cfg.per_cu, s, scratch);
}

int64_t bf16x3_blocks(int cfg, int64_t M, int64_t N) {
  const auto& c = bf16x3_table().at(cfg).cfg;
  return ((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
}

}  // namespace qp

// Quaternion GEMM with BF16 operands on gfx950 MFMA (v_mfma_f32_16x16x32_bf16), FP32 storage and
// FP32 accumulation: the early, self-correcting iterations of the precision ladder.
//
// The operand planes stay FP32 in HBM; each workgroup rounds them to BF16 (round to nearest even)
// while staging into LDS, so no BF16 copy of any matrix exists.  LDS holds A tiles as [plane][row][k]
// and B tiles transposed as [plane][col][k], both k-contiguous, so that every lane reads its eight
// consecutive k of a fragment with one 16-byte LDS load.  Lane layout (64 lanes, verified):
//   A frag: row l%16, k = 8(l/16) .. 8(l/16)+7;  B frag: col l%16, same k;  D reg r: row 4(l/16)+r, col l%16.
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

struct Bf16Entry {
  TileConfig cfg;
  int64_t (*fn)(const GemmParams<float>&, int, hipStream_t);
};

static const std::vector<Bf16Entry>& bf16_table() {
  static const std::vector<Bf16Entry> t = {
      {{0, 64, 64, 32, 256, "bf16_64x64x32_w2x2_mfma16x16x32"}, launch_bf16<64, 64, 2, 2>},
      {{1, 32, 32, 32, 256, "bf16_32x32x32_w2x2_mfma16x16x32"}, launch_bf16<32, 32, 2, 2>},
      {{2, 128, 64, 32, 256, "bf16_128x64x32_w2x2_mfma16x16x32"}, launch_bf16<128, 64, 2, 2>},
      {{3, 64, 128, 32, 256, "bf16_64x128x32_w2x2_mfma16x16x32"}, launch_bf16<64, 128, 2, 2>},
      {{4, 32, 32, 32, 256, "bf16_32x32x32_w2x2_mfma16x16x32_cu3", 3}, launch_bf16<32, 32, 2, 2>},
      {{5, 64, 64, 32, 256, "bf16_64x64x32_w2x2_mfma16x16x32_cu2", 2}, launch_bf16<64, 64, 2, 2>},
  };
  return t;
}

const std::vector<TileConfig>& bf16_configs() {
  static std::vector<TileConfig> v;
  if (v.empty())
    for (auto& e : bf16_table()) v.push_back(e.cfg);
  return v;
}

int64_t bf16_launch(const GemmParams<float>& P, int cfg, hipStream_t s) {
  const auto& e = bf16_table().at(cfg);
  return e.fn(P, e.cfg.per_cu, s);
}

int64_t bf16_blocks(int cfg, int64_t M, int64_t N) {
  const auto& c = bf16_table().at(cfg).cfg;
  return ((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
}

}  // namespace qp

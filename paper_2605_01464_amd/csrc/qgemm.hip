// Quaternion GEMM kernels for gfx950 (CDNA4): FP32 and FP64 MFMA, with fused epilogues.
//
// Work decomposition
//   * one workgroup computes a BM x BN tile of all four output planes;
//   * per K-step of BK it stages the four A planes (BM x BK, stored k-major so that a fragment
//     read is 32/16 consecutive words) and the four B planes (BK x BN) in LDS, prefetching the
//     next K-step into registers while the MFMAs run on the current one;
//   * each wave owns a (BM/WM) x (BN/WN) sub-tile as MFMA blocks; for every fragment set it issues
//     the 16 signed plane products of the Hamilton product (a sign flip of an A fragment is one
//     VALU op, so the 4x-expanded real representation never exists anywhere);
//   * the epilogue applies up to three output combinations and optional reductions.
// Block ids are remapped so that the workgroups resident on one XCD (the hardware deals ids
// round-robin over the 8 XCDs) take neighbouring tiles, grouped 8 tile-rows at a time, to share
// that XCD's L2.
#include <algorithm>
#include <vector>

#include "qgemm_kern.hpp"

namespace qp {

template <class MM, int BM, int BN, int BK, int WM, int WN, int FLUSH>
__global__ void __launch_bounds__(64 * WM * WN) qgemm_kernel(GemmParams<typename MM::T> P) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  __shared__ typename MM::T smem[C::SMEM];
  __shared__ double red_lds[C::NW][2];
  int tm, tn;
  tile_of_block(blockIdx.x, P.tiles_m * P.tiles_n, P.tiles_m, P.tiles_n, tm, tn);
  double s_d = 0.0, s_x = 0.0;
  gemm_tile<MM, BM, BN, BK, WM, WN, FLUSH>(P, tm, tn, smem, s_d, s_x);
  store_partials<C::NW>(P.partial, s_d, s_x, red_lds, threadIdx.x & 63, threadIdx.x >> 6, threadIdx.x);
}

// Deterministic sum of `count` (d, x) pairs: one workgroup, fixed strided order, fixed tree.
__global__ void __launch_bounds__(256) reduce_pairs_kernel(const double* __restrict__ partial, int64_t count,
                                                           double* __restrict__ red) {
  __shared__ double s0[256], s1[256];
  double a0 = 0.0, a1 = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) {
    a0 += partial[2 * i];
    a1 += partial[2 * i + 1];
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[0] = s0[0];
    red[1] = s1[0];
  }
}

void reduce_pairs(const double* partial, int64_t count, double* red, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_pairs_kernel, dim3(1), dim3(256), 0, stream, partial, count, red);
  QP_HIP(hipGetLastError());
}

// ------------------------------------------------------------------------------------------------
// configuration table and dispatch
// ------------------------------------------------------------------------------------------------
template <class MM, int BM, int BN, int BK, int WM, int WN, int FLUSH>
static void launch_cfg(const GemmParams<typename MM::T>& P0, hipStream_t s) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  GemmParams<typename MM::T> P = P0;
  P.tiles_m = (P.M + BM - 1) / BM;
  P.tiles_n = (P.N + BN - 1) / BN;
  const int nb = P.tiles_m * P.tiles_n;
  if (nb == 0) return;
  hipLaunchKernelGGL((qgemm_kernel<MM, BM, BN, BK, WM, WN, FLUSH>), dim3(nb), dim3(C::NT), 0, s, P);
  QP_HIP(hipGetLastError());
}

using F32Launch = void (*)(const GemmParams<float>&, hipStream_t);
using F64Launch = void (*)(const GemmParams<double>&, hipStream_t);

struct F32Entry {
  TileConfig cfg;
  F32Launch fn;
};
struct F64Entry {
  TileConfig cfg;
  F64Launch fn;
};

// FP32 configurations accumulate in two levels (flush every 128 k); FP64 needs no flush.
static const std::vector<F32Entry>& f32_table() {
  static const std::vector<F32Entry> t = {
      {{0, 64, 64, 16, 256, "f32_64x64x16_w2x2_mfma32"}, launch_cfg<MM32F, 64, 64, 16, 2, 2, 128>},
      {{1, 32, 32, 16, 256, "f32_32x32x16_w2x2_mfma16"}, launch_cfg<MM16F, 32, 32, 16, 2, 2, 128>},
      {{2, 128, 64, 16, 256, "f32_128x64x16_w2x2_mfma32"}, launch_cfg<MM32F, 128, 64, 16, 2, 2, 128>},
      {{3, 64, 128, 16, 256, "f32_64x128x16_w2x2_mfma32"}, launch_cfg<MM32F, 64, 128, 16, 2, 2, 128>},
      {{4, 64, 64, 16, 256, "f32_64x64x16_w2x2_mfma16"}, launch_cfg<MM16F, 64, 64, 16, 2, 2, 128>},
  };
  return t;
}

static const std::vector<F64Entry>& f64_table() {
  static const std::vector<F64Entry> t = {
      {{0, 64, 64, 8, 256, "f64_64x64x8_w2x2_mfma16"}, launch_cfg<MM16D, 64, 64, 8, 2, 2, 0>},
      {{1, 32, 32, 16, 256, "f64_32x32x16_w2x2_mfma16"}, launch_cfg<MM16D, 32, 32, 16, 2, 2, 0>},
      {{2, 64, 64, 8, 1024, "f64_64x64x8_w4x4_mfma16"}, launch_cfg<MM16D, 64, 64, 8, 4, 4, 0>},
  };
  return t;
}

const std::vector<TileConfig>& bf16_configs();  // qgemm_bf16.hip

const std::vector<TileConfig>& tile_configs(Prec p) {
  static std::vector<TileConfig> f32, f64;
  if (f32.empty()) {
    for (auto& e : f32_table()) f32.push_back(e.cfg);
    for (auto& e : f64_table()) f64.push_back(e.cfg);
  }
  if (p == P_BF16) return bf16_configs();
  return p == P_F64 ? f64 : f32;
}

static int64_t blocks_for(const TileConfig& c, int64_t M, int64_t N) {
  return ((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
}

int64_t qgemm_blocks(Prec p, int cfg, int64_t M, int64_t N) {
  const auto& t = tile_configs(p);
  return blocks_for(t.at(cfg), M, N);
}

int default_config(Prec p, int64_t M, int64_t N, int64_t K) {
  (void)K;
  if (p == P_F64) {
    return blocks_for(tile_configs(p)[0], M, N) >= 256 ? 0 : 1;
  }
  const auto& t = tile_configs(p);
  if (p == P_BF16) return blocks_for(t[0], M, N) >= 256 ? 0 : 1;
  return blocks_for(t[0], M, N) >= 512 ? 0 : 1;
}

template <class T>
static GemmParams<T> make_params(const QView& A, const QView& B, int64_t M, int64_t N, int64_t K,
                                 const Epilogue& e, double* partial) {
  GemmParams<T> P{};
  P.A = static_cast<const T*>(A.p);
  P.lda = A.ld;
  P.psa = A.ps;
  P.B = static_cast<const T*>(B.p);
  P.ldb = B.ld;
  P.psb = B.ps;
  P.M = (int)M;
  P.N = (int)N;
  P.K = (int)K;
  P.nout = e.nout;
  P.nin = e.nin;
  P.ref = e.ref;
  constexpr int VA = V16<T>::n;
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  P.vec = al(A.p) && al(B.p) && A.ld % VA == 0 && B.ld % VA == 0 && A.ps % VA == 0 && B.ps % VA == 0;
  for (int t = 0; t < 3; ++t) {
    P.out[t] = t < e.nout ? static_cast<T*>(e.out[t].p) : nullptr;
    P.ldo[t] = e.out[t].ld;
    P.pso[t] = e.out[t].ps;
    P.in[t] = t < e.nin ? static_cast<const T*>(e.in[t].p) : nullptr;
    P.ldi[t] = e.in[t].ld;
    P.psi[t] = e.in[t].ps;
    P.ca[t] = (T)e.a[t];
    P.cg[t] = (T)e.g[t];
    for (int u = 0; u < 3; ++u) P.cb[t][u] = (T)e.b[t][u];
  }
  P.partial = e.reduce ? partial : nullptr;
  P.reduce = e.reduce ? 1 : 0;
  return P;
}

void bf16_launch(const GemmParams<float>& P, int cfg, hipStream_t s);  // qgemm_bf16.hip
int64_t bf16_blocks(int cfg, int64_t M, int64_t N);

void qgemm(Prec p, const QView& A, const QView& B, int64_t M, int64_t N, int64_t K, const Epilogue& epi,
           double* red, GemmScratch& scratch, hipStream_t stream, int cfg) {
  if (M < 0 || N < 0 || K < 0) throw Error(-1, "qgemm: negative size");
  if (epi.nout < 1 || epi.nout > 3 || epi.nin < 0 || epi.nin > 3) throw Error(-1, "qgemm: bad epilogue");
  if (epi.reduce && (!red || epi.ref >= epi.nin)) throw Error(-1, "qgemm: bad reduction");
  if (cfg < 0) cfg = default_config(p, M, N, K);
  const auto& cfgs = tile_configs(p);
  if (cfg >= (int)cfgs.size()) throw Error(-1, "qgemm: bad tile config");
  const int64_t nb = p == P_BF16 ? bf16_blocks(cfg, M, N) : blocks_for(cfgs[cfg], M, N);
  if (epi.reduce && nb > scratch.capacity / 2) throw Error(-1, "qgemm: reduction scratch too small");
  double* partial = epi.reduce ? scratch.partial : nullptr;
  if (p == P_F64) {
    f64_table()[cfg].fn(make_params<double>(A, B, M, N, K, epi, partial), stream);
  } else if (p == P_F32) {
    f32_table()[cfg].fn(make_params<float>(A, B, M, N, K, epi, partial), stream);
  } else {
    bf16_launch(make_params<float>(A, B, M, N, K, epi, partial), cfg, stream);
  }
  if (epi.reduce) reduce_pairs(partial, nb, red, stream);
}

}  // namespace qp

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
#include <mutex>
#include <vector>

#include "qgemm_kern.hpp"

namespace qp {

// A workgroup computes tiles blockIdx.x, blockIdx.x + gridDim.x, ... (one tile when the grid covers
// them all).  With a grid that is a multiple of 8, every tile a workgroup visits maps to the same XCD
// range, so the XCD-aware order is kept.
// WALK = false: one tile per workgroup.  WALK = true: tiles blockIdx.x, blockIdx.x + gridDim.x, ...
// (a separate instantiation, so that the loop's live state does not raise the register count, and
// with it lower the occupancy, of the one-tile form).  With a grid that is a multiple of 8, every tile a
// workgroup visits maps to the same XCD range, so the XCD-aware order is kept.  LM (the operand load
// mode) and DB as in gemm_tile.
template <class MM, int BM, int BN, int BK, int WM, int WN, int FLUSH, bool DB, int LM, bool WALK, int MINW>
__global__ void __launch_bounds__(64 * WM * WN, MINW) qgemm_kernel(GemmParams<typename MM::T> P) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) typename MM::T smem[DB ? 2 * C::SMEM : C::SMEM];
  __shared__ double red_lds[C::NW][2];
  const int nt = P.tiles_m * P.tiles_n;
  double s_d = 0.0, s_x = 0.0;
  if constexpr (WALK) {
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
      int tm, tn;
      tile_of_block(t, nt, P.tiles_m, P.tiles_n, tm, tn);
      gemm_tile<MM, BM, BN, BK, WM, WN, FLUSH, LM, DB>(P, tm, tn, smem, s_d, s_x);
    }
  } else {
    int tm, tn;
    tile_of_block(blockIdx.x, nt, P.tiles_m, P.tiles_n, tm, tn);
    gemm_tile<MM, BM, BN, BK, WM, WN, FLUSH, LM, DB>(P, tm, tn, smem, s_d, s_x);
  }
  store_partials<C::NW>(P.partial, s_d, s_x, red_lds, threadIdx.x & 63, threadIdx.x >> 6, threadIdx.x);
}

namespace {
struct DevLimits {
  int cus = 0;
  int lds = 0;  // bytes of LDS per compute unit
};

DevLimits dev_limits() {
  static std::mutex mu;
  static std::vector<DevLimits> cache;
  int dev = 0;
  QP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1);
  DevLimits& d = cache[dev];
  if (d.cus == 0) {
    QP_HIP(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
    QP_HIP(hipDeviceGetAttribute(&d.lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
  }
  return d;
}
}  // namespace

LaunchShape launch_shape(int64_t tiles, int per_cu, int occ, size_t static_lds) {
  LaunchShape ls;
  ls.grid = tiles;
  if (per_cu <= 0 || tiles == 0) return ls;
  const DevLimits d = dev_limits();
  const int c = std::max(1, std::min(per_cu, occ));
  int64_t cap = (int64_t)d.cus * c;
  if (cap >= 8) cap &= ~(int64_t)7;
  if (tiles <= cap) return ls;
  ls.grid = cap;
  // reserve LDS so that at most c workgroups fit on a compute unit (kept within the 64 KiB a
  // workgroup may take without opting in)
  if (d.lds > 0) {
    const size_t target = (size_t)((double)d.lds / (c + 0.5));
    if (target > static_lds) ls.dyn_lds = std::min<size_t>(target, 65536) - static_lds;
  }
  return ls;
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
// Resident workgroups per compute unit and static LDS bytes of a kernel (queried once).
struct KernelLimits {
  int occ = 1;
  size_t lds = 0;
};

template <class K>
static KernelLimits kernel_limits(K kern, int threads) {
  KernelLimits k;
  int occ = 0;
  QP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, 0));
  hipFuncAttributes fa{};
  QP_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)));
  k.occ = std::max(occ, 1);
  k.lds = fa.sharedSizeBytes;
  return k;
}

// Launches the configuration; returns the number of workgroups (partial sums) launched.  PER_CU as
// TileConfig::per_cu.  The operand load mode is the most specific one the shape and the views allow.
// MINW: waves per SIMD the register allocation must leave room for (launch bound).
template <class MM, int BM, int BN, int BK, int WM, int WN, int FLUSH, bool DB, int MINW, bool WALK, int LM>
static void launch_mode(const GemmParams<typename MM::T>& P, int64_t grid, size_t dyn_lds, hipStream_t s) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  hipLaunchKernelGGL((qgemm_kernel<MM, BM, BN, BK, WM, WN, FLUSH, DB, LM, WALK, MINW>), dim3((unsigned)grid), dim3(C::NT),
                     dyn_lds, s, P);
}

template <class MM, int BM, int BN, int BK, int WM, int WN, int FLUSH, bool DB, int MINW, bool WALK>
static void launch_any_mode(const GemmParams<typename MM::T>& P, int64_t grid, size_t dyn_lds, hipStream_t s) {
  if (P.vec && P.M % BM == 0 && P.N % BN == 0 && P.K % BK == 0)
    launch_mode<MM, BM, BN, BK, WM, WN, FLUSH, DB, MINW, WALK, kLoadAligned>(P, grid, dyn_lds, s);
  else if (P.vec)
    launch_mode<MM, BM, BN, BK, WM, WN, FLUSH, DB, MINW, WALK, kLoadVec>(P, grid, dyn_lds, s);
  else
    launch_mode<MM, BM, BN, BK, WM, WN, FLUSH, DB, MINW, WALK, kLoadScalar>(P, grid, dyn_lds, s);
  QP_HIP(hipGetLastError());
}

template <class MM, int BM, int BN, int BK, int WM, int WN, int FLUSH, bool DB, int PER_CU, int MINW = 1>
static int64_t launch_cfg(const GemmParams<typename MM::T>& P0, hipStream_t s) {
  using C = GemmCfg<MM, BM, BN, BK, WM, WN>;
  GemmParams<typename MM::T> P = P0;
  P.tiles_m = (P.M + BM - 1) / BM;
  P.tiles_n = (P.N + BN - 1) / BN;
  const int64_t nt = (int64_t)P.tiles_m * P.tiles_n;
  if (nt == 0) return 0;
  if constexpr (PER_CU > 0) {
    static const KernelLimits kl =
        kernel_limits(qgemm_kernel<MM, BM, BN, BK, WM, WN, FLUSH, DB, kLoadAligned, true, MINW>, C::NT);
    const LaunchShape ls = launch_shape(nt, PER_CU, kl.occ, kl.lds);
    if (ls.grid < nt) {
      launch_any_mode<MM, BM, BN, BK, WM, WN, FLUSH, DB, MINW, true>(P, ls.grid, ls.dyn_lds, s);
      return ls.grid;
    }
  }
  launch_any_mode<MM, BM, BN, BK, WM, WN, FLUSH, DB, MINW, false>(P, nt, 0, s);
  return nt;
}

using F32Launch = int64_t (*)(const GemmParams<float>&, hipStream_t);
using F64Launch = int64_t (*)(const GemmParams<double>&, hipStream_t);

struct F32Entry {
  TileConfig cfg;
  F32Launch fn;
};
struct F64Entry {
  TileConfig cfg;
  F64Launch fn;
};

// FP32 configurations accumulate in two levels (flush every 128 k); FP64 needs no flush.
// "_db": double-buffered LDS staging; "_cuC": C workgroups per compute unit walking the tiles.
static const std::vector<F32Entry>& f32_table() {
  static const std::vector<F32Entry> t = {
      {{0, 64, 64, 16, 256, "f32_64x64x16_w2x2_mfma32"}, launch_cfg<MM32F, 64, 64, 16, 2, 2, 128, false, 0>},
      {{1, 32, 32, 16, 256, "f32_32x32x16_w2x2_mfma16"}, launch_cfg<MM16F, 32, 32, 16, 2, 2, 128, false, 0>},
      {{2, 128, 64, 16, 256, "f32_128x64x16_w2x2_mfma32"}, launch_cfg<MM32F, 128, 64, 16, 2, 2, 128, false, 0>},
      {{3, 64, 128, 16, 256, "f32_64x128x16_w2x2_mfma32"}, launch_cfg<MM32F, 64, 128, 16, 2, 2, 128, false, 0>},
      {{4, 64, 64, 16, 256, "f32_64x64x16_w2x2_mfma16"}, launch_cfg<MM16F, 64, 64, 16, 2, 2, 128, false, 0>},
      {{5, 64, 64, 16, 256, "f32_64x64x16_w2x2_mfma32_db"}, launch_cfg<MM32F, 64, 64, 16, 2, 2, 128, true, 0>},
      {{6, 32, 32, 16, 256, "f32_32x32x16_w2x2_mfma16_db"}, launch_cfg<MM16F, 32, 32, 16, 2, 2, 128, true, 0>},
      {{7, 64, 64, 16, 1024, "f32_64x64x16_w4x4_mfma16_db"}, launch_cfg<MM16F, 64, 64, 16, 4, 4, 128, true, 0>},
      {{8, 32, 32, 16, 256, "f32_32x32x16_w2x2_mfma16_db_cu3", 3}, launch_cfg<MM16F, 32, 32, 16, 2, 2, 128, true, 3>},
  };
  return t;
}

static const std::vector<F64Entry>& f64_table() {
  static const std::vector<F64Entry> t = {
      {{0, 64, 64, 8, 256, "f64_64x64x8_w2x2_mfma16"}, launch_cfg<MM16D, 64, 64, 8, 2, 2, 0, false, 0>},
      {{1, 32, 32, 16, 256, "f64_32x32x16_w2x2_mfma16"}, launch_cfg<MM16D, 32, 32, 16, 2, 2, 0, false, 0>},
      {{2, 64, 64, 8, 1024, "f64_64x64x8_w4x4_mfma16"}, launch_cfg<MM16D, 64, 64, 8, 4, 4, 0, false, 0>},
      {{3, 32, 32, 16, 256, "f64_32x32x16_w2x2_mfma16_db"}, launch_cfg<MM16D, 32, 32, 16, 2, 2, 0, true, 0>},
      {{4, 64, 64, 8, 1024, "f64_64x64x8_w4x4_mfma16_db"}, launch_cfg<MM16D, 64, 64, 8, 4, 4, 0, true, 0>},
      {{5, 128, 64, 8, 512, "f64_128x64x8_w4x2_mfma16_db"}, launch_cfg<MM16D, 128, 64, 8, 4, 2, 0, true, 0>},
      {{6, 64, 128, 8, 512, "f64_64x128x8_w2x4_mfma16_db"}, launch_cfg<MM16D, 64, 128, 8, 2, 4, 0, true, 0>},
  };
  return t;
}

const std::vector<TileConfig>& bf16_configs();    // qgemm_bf16.hip
const std::vector<TileConfig>& bf16x3_configs();  // qgemm_bf16.hip

const std::vector<TileConfig>& tile_configs(Prec p) {
  static std::vector<TileConfig> f32, f64;
  if (f32.empty()) {
    for (auto& e : f32_table()) f32.push_back(e.cfg);
    for (auto& e : f64_table()) f64.push_back(e.cfg);
  }
  if (p == P_BF16) return bf16_configs();
  if (p == P_BF16X3) return bf16x3_configs();
  return p == P_F64 ? f64 : f32;
}

static int64_t blocks_for(const TileConfig& c, int64_t M, int64_t N) {
  return ((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
}

int64_t qgemm_blocks(Prec p, int cfg, int64_t M, int64_t N) {
  const auto& t = tile_configs(p);
  return blocks_for(t.at(cfg), M, N);
}

// Measured on MI355X: the 64 x 64 double-buffered tiles win once there are >= 4 of them per compute unit,
// the 32 x 32 ones below that (fewer tiles leave compute units idle in the last wave); for FP64 the 64 x 128
// double-buffered tiles (8 waves of 32 x 32, twice the MFMA work per K-step barrier) beat 64 x 64 there
// (4096^3: 30.8 vs 31.3 ms; 128 x 64 with the same waves 36.6 ms).  BF16 from 1024 tiles
// of 64 x 64: the staged form with its operand tiles loaded straight into LDS; split BF16: 128 x 128 tiles
// from 256 of them (one workgroup of 16 waves per CU), 64 x 64 below.
int default_config(Prec p, int64_t M, int64_t N, int64_t K) {
  (void)K;
  const int64_t b64 = ((M + 63) / 64) * ((N + 63) / 64);
  if (p == P_F64) return b64 >= 1024 ? 6 : 1;
  if (p == P_BF16) return b64 >= 1024 ? 11 : b64 >= 256 ? 0 : 1;
  if (p == P_BF16X3) return ((M + 127) / 128) * ((N + 127) / 128) >= 256 ? 4 : 3;
  return b64 >= 1024 ? 5 : 6;
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

int64_t bf16_launch(const GemmParams<float>& P, int cfg, hipStream_t s, GemmScratch& scratch);  // qgemm_bf16.hip
int64_t bf16_blocks(int cfg, int64_t M, int64_t N);
int64_t bf16x3_launch(const GemmParams<float>& P, int cfg, hipStream_t s, GemmScratch& scratch);
int64_t bf16x3_blocks(int cfg, int64_t M, int64_t N);

void qgemm(Prec p, const QView& A, const QView& B, int64_t M, int64_t N, int64_t K, const Epilogue& epi,
           double* red, GemmScratch& scratch, hipStream_t stream, int cfg) {
  if (M < 0 || N < 0 || K < 0) throw Error(-1, "qgemm: negative size");
  if (epi.nout < 1 || epi.nout > 3 || epi.nin < 0 || epi.nin > 3) throw Error(-1, "qgemm: bad epilogue");
  if (epi.reduce && (!red || epi.ref >= epi.nin)) throw Error(-1, "qgemm: bad reduction");
  if (cfg < 0) cfg = default_config(p, M, N, K);
  const auto& cfgs = tile_configs(p);
  if (cfg >= (int)cfgs.size()) throw Error(-1, "qgemm: bad tile config");
  // an upper bound of the workgroups launched (a per-CU configuration launches at most this many)
  const int64_t nb = p == P_BF16     ? bf16_blocks(cfg, M, N)
                     : p == P_BF16X3 ? bf16x3_blocks(cfg, M, N)
                                     : blocks_for(cfgs[cfg], M, N);
  if (epi.reduce && nb > scratch.capacity / 2) throw Error(-1, "qgemm: reduction scratch too small");
  double* partial = epi.reduce ? scratch.partial : nullptr;
  int64_t launched = 0;
  if (p == P_F64) {
    launched = f64_table()[cfg].fn(make_params<double>(A, B, M, N, K, epi, partial), stream);
  } else if (p == P_F32) {
    launched = f32_table()[cfg].fn(make_params<float>(A, B, M, N, K, epi, partial), stream);
  } else if (p == P_BF16) {
    launched = bf16_launch(make_params<float>(A, B, M, N, K, epi, partial), cfg, stream, scratch);
  } else {
    launched = bf16x3_launch(make_params<float>(A, B, M, N, K, epi, partial), cfg, stream, scratch);
  }
  if (epi.reduce) reduce_pairs(partial, launched, red, stream);
}

}  // namespace qp

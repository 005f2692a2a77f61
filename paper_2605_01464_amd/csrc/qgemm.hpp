// Quaternion GEMM with a fused multi-output epilogue (host interface).
//
// C = A B for quaternion matrices (Hamilton product, Section 2).  In real form the four output
// planes are [C_s C_x C_y C_z] = [A_s A_x A_y A_z] Rrep(B), where Rrep(B) is the 4x4 block matrix of
// signed B planes; one quaternion product of shape (M x K)(K x N) is 32 M K N real flops.  The
// kernels never build Rrep(B): each workgroup stages the four planes of an A tile and a B tile in
// LDS and issues the 16 signed plane products on MFMA.
//
// The epilogue writes up to three outputs of shape M x N, each
//     out_t = a_t (A B) + sum_u b_tu in_u + g_t I
// (I = quaternion identity: ones on the diagonal of the real plane), and can reduce
// sum |out_0 - in_ref|^2 and sum |out_0|^2 (for the change ||X_{j+1} - X_j||_F of an update).
#pragma once

#include <vector>

#include "common.hpp"

namespace qp {

// P_BF16X3: FP32 storage, each product as three BF16 products of split operands (hi.hi + hi.lo + lo.hi)
enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3 };

struct Epilogue {
  int nout = 1;
  QView out[3];
  double a[3] = {1.0, 1.0, 1.0};
  int nin = 0;
  QView in[3];
  double b[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double g[3] = {0.0, 0.0, 0.0};
  bool reduce = false;
  int ref = -1;  // input compared with out_0 in the reduction (-1: none)
};

// Per-stream scratch for the epilogue reduction (per-workgroup partial sums).
struct GemmScratch {
  double* partial = nullptr;  // device, capacity doubles
  int64_t capacity = 0;
  void* stage = nullptr;  // device, stage_bytes: BF16 operand copies of the staged BF16 products (grown on
  size_t stage_bytes = 0;  // demand, outside graph capture; owned and freed by the context)
  bool no_grow = false;    // allocation-free call: a product that needs a larger stage buffer fails instead
};

struct TileConfig {
  int id;
  int bm, bn, bk, threads;
  const char* name;
  int per_cu = 0;  // 0: one workgroup per output tile.  c > 0: c workgroups per compute unit (LDS
                   // reservation caps residency at c) each walking an equal share of the tiles, so
                   // tile counts that are a multiple of c x CUs finish without a partial last wave
};

// Launch geometry of a configuration on the current device: workgroups launched and the dynamic LDS
// reservation that caps residency.
struct LaunchShape {
  int64_t grid = 0;
  size_t dyn_lds = 0;
};

// Workgroups and dynamic LDS for `tiles` output tiles of a kernel with `static_lds` bytes of LDS,
// `occ` resident workgroups per compute unit, `per_cu` as in TileConfig.
LaunchShape launch_shape(int64_t tiles, int per_cu, int occ, size_t static_lds);

// Tile configurations available for a compute precision (F32/BF16 take float storage,
// F64 takes double storage).
const std::vector<TileConfig>& tile_configs(Prec p);

// Heuristic choice of tile configuration for a shape (used when no tuned choice exists).
int default_config(Prec p, int64_t M, int64_t N, int64_t K);

// Launch C = A B with the epilogue.  A is M x K, B is K x N, outputs/inputs M x N.
// If epi.reduce, `red` (device, 2 doubles) receives {sum |out0 - in_ref|^2, sum |out0|^2}.
// cfg < 0 selects the default configuration.
void qgemm(Prec p, const QView& A, const QView& B, int64_t M, int64_t N, int64_t K, const Epilogue& epi,
           double* red, GemmScratch& scratch, hipStream_t stream, int cfg = -1);

// Number of workgroups a configuration launches for an M x N output (sizes scratch).
int64_t qgemm_blocks(Prec p, int cfg, int64_t M, int64_t N);
// whether a P_BF16X3 product of this shape fits the split copies' 32-bit buffer offsets
bool bf16x3_fits(int64_t M, int64_t N, int64_t K);

// Sum `count` pairs of partial sums at `partial` into red[0..1] (fixed order, deterministic).
void reduce_pairs(const double* partial, int64_t count, double* red, hipStream_t stream);

}  // namespace qp

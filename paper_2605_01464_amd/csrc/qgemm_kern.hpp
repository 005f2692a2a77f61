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
template <>
struct V16<float> {
  using type = float4;
  static constexpr int n = 4;
};
template <>
struct V16<double> {
  using type = double2;
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
  double* partial;
};

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


// out_t = a_t v + sum_u b_tu in_u + g_t I for plane p at one element, plus the reduction terms.
template <class T>
__device__ __forceinline__ void epilogue_plane(const GemmParams<T>& P, int p, int row, int col, T v, double& s_d,
                                               double& s_x) {
  if (row >= P.M || col >= P.N) return;
  T inv[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) inv[u] = (u < P.nin) ? P.in[u][p * P.psi[u] + (int64_t)row * P.ldi[u] + col] : T(0);
  const T eye = (p == 0 && row == col) ? T(1) : T(0);
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t < P.nout) {
      const T o = P.ca[t] * v + P.cg[t] * eye + P.cb[t][0] * inv[0] + P.cb[t][1] * inv[1] + P.cb[t][2] * inv[2];
      P.out[t][p * P.pso[t] + (int64_t)row * P.ldo[t] + col] = o;
      if (t == 0 && P.partial) {
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

}  // namespace qp

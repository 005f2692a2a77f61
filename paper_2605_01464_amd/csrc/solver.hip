// Solver driver: the method chains of Section 3 as sequences of fused quaternion products, the
// scaling step, the stop-rule controller and the precision phases.
//
// Residual side.  The paper forms R_j = I_m - A X_j (m x m).  The push-through identity
// X p(A X) = p(X A) X (true for every polynomial p) gives the same iterate from R'_j = I_n - X_j A
// (n x n).  Side LEFT uses I_n - X A and X_{j+1} = p(R') X; side RIGHT uses I_m - A X and
// X_{j+1} = X p(R).  AUTO takes the smaller of m and n, which is where all the s^3 products live.
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>

#include "aux.hpp"
#include "batched.hpp"
#include "controller.hpp"
#include "mlp.hpp"
#include "solver.hpp"

namespace qp {

// ------------------------------------------------------------------------------------------------
// coefficients from their closed forms
//   QSAI: beta_{1,2} = (1 +- sqrt 5)/2 (Section 3, QSAI).
//   QHPI19: d_1, d_2 = (1 +- sqrt(27 - 2 sqrt 93))/4, d_3 = (5 sqrt 93 - 93)/496,
//           e_1 = (-93 - 5 sqrt 93)/496, e_2 = -sqrt(93)/4, c_1 = 3/8, c_2 = 321/1984
//           (Section 3, QHPI19: polynomial and secondary factorization).
// ------------------------------------------------------------------------------------------------
namespace {
const double kS5 = std::sqrt(5.0);
const double kBeta1 = 0.5 * (1.0 + kS5);
const double kBeta2 = 0.5 * (1.0 - kS5);
const double kS93 = std::sqrt(93.0);
const double kRt = std::sqrt(27.0 - 2.0 * kS93);
const double kD1 = 0.25 * (1.0 + kRt);
const double kD2 = 0.25 * (1.0 - kRt);
const double kD3 = (5.0 * kS93 - 93.0) / 496.0;
const double kE1 = (-93.0 - 5.0 * kS93) / 496.0;
const double kE2 = -0.25 * kS93;
const double kC1 = 3.0 / 8.0;
const double kC2 = 321.0 / 1984.0;

inline int store_of(Prec p) { return p == P_F64 ? QPINV_F64 : QPINV_F32; }
inline size_t esize(int dtype) { return dtype == QPINV_F64 ? 8 : 4; }
inline int64_t round8(int64_t x) { return (x + 7) / 8 * 8; }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

Epilogue epi1(const Mat& o, double a = 1.0, double g = 0.0) {
  Epilogue e;
  e.nout = 1;
  e.out[0] = o.v;
  e.a[0] = a;
  e.g[0] = g;
  return e;
}
}  // namespace

// ------------------------------------------------------------------------------------------------
// workspace / context
// ------------------------------------------------------------------------------------------------
void* Workspace::get(const std::string& key, size_t bytes) {
  if (bytes < 256) bytes = 256;
  if (arena) {
    auto it = arena_bufs.find(key);
    if (it != arena_bufs.end() && it->second.bytes >= bytes) return it->second.p;
    bytes = (bytes + 255) / 256 * 256;
    if (bytes > arena_cap - arena_used)
      throw Error(QPINV_EINVAL, "allocation-free solve: workspace request " + key + " of " + std::to_string(bytes) +
                                    " bytes does not fit the " + std::to_string(arena_cap) + "-byte scratch (" +
                                    std::to_string(arena_used) + " bytes in use)");
    void* p = arena + arena_used;
    arena_used += bytes;
    arena_bufs[key] = Buf{p, bytes};
    return p;
  }
  auto it = bufs.find(key);
  if (it != bufs.end() && it->second.bytes >= bytes) return it->second.p;
  if (it != bufs.end()) {
    (void)hipFree(it->second.p);
    bufs.erase(it);
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(QPINV_ENOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed (" + key + ")");
  }
  bufs[key] = Buf{p, bytes};
  return p;
}

void Workspace::begin_arena(void* base, size_t cap) {
  arena = static_cast<char*>(base);
  arena_cap = cap;
  arena_used = 0;
  arena_bufs.clear();
}

void Workspace::end_arena() {
  arena = nullptr;
  arena_cap = arena_used = 0;
  arena_bufs.clear();
}

void Workspace::release() {
  for (auto& kv : bufs) (void)hipFree(kv.second.p);
  bufs.clear();
}

Ctx::Ctx(int dev) : device(dev) {
  QP_HIP(hipSetDevice(dev));
  scratch.capacity = 1 << 20;
  QP_HIP(hipMalloc(&scratch.partial, sizeof(double) * scratch.capacity));
  QP_HIP(hipMalloc(&dsc, sizeof(double) * 64));
  QP_HIP(hipHostMalloc(&hsc, sizeof(double) * 64, hipHostMallocDefault));
  QP_HIP(hipHostMalloc(&hstage, kStageBytes, hipHostMallocDefault));
  (void)noalloc_scratch(dev);  // look up this device's no-allocation scratch now, with the device current
}

Ctx::~Ctx() {
  (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  for (auto& e : events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  delete batched;
  ws.release();
  if (scratch.partial) (void)hipFree(scratch.partial);
  if (scratch.stage) (void)hipFree(scratch.stage);
  if (dsc) (void)hipFree(dsc);
  if (hsc) (void)hipHostFree(hsc);
  if (hstage) (void)hipHostFree(hstage);
}

int Ctx::config_for(Prec p, int64_t M, int64_t N, int64_t K, hipStream_t s) {
  if (opt.force_cfg[(int)p] >= 0) return opt.force_cfg[(int)p];
  auto key = std::make_tuple((int)p, M, N, K);
  auto it = tuned.find(key);
  if (it != tuned.end()) return it->second;
  if (opt.autotune && !no_alloc) return autotune(*this, p, M, N, K, nullptr, s);
  return default_config(p, M, N, K);
}

Mat from_abi(const qpinv_qmat& q) {
  Mat m;
  m.v.p = q.data;
  m.v.rows = q.rows;
  m.v.cols = q.cols;
  m.v.ld = q.ld;
  m.v.ps = q.plane_stride;
  m.rows = q.rows;
  m.cols = q.cols;
  m.dtype = q.dtype;
  return m;
}

void validate(const qpinv_qmat* q, const char* what) {
  if (!q) throw Error(QPINV_EINVAL, std::string(what) + ": null descriptor");
  if (q->dtype != QPINV_F32 && q->dtype != QPINV_F64) throw Error(QPINV_EINVAL, std::string(what) + ": bad dtype");
  if (q->rows < 0 || q->cols < 0) throw Error(QPINV_EINVAL, std::string(what) + ": negative shape");
  if (q->rows > (1 << 20) || q->cols > (1 << 20)) throw Error(QPINV_EINVAL, std::string(what) + ": shape too large");
  if (q->ld < q->cols || q->ld < 1) throw Error(QPINV_EINVAL, std::string(what) + ": ld < cols");
  if (q->plane_stride < q->rows * q->ld) throw Error(QPINV_EINVAL, std::string(what) + ": plane_stride < rows*ld");
  if (q->rows > 0 && q->cols > 0 && !q->data) throw Error(QPINV_EINVAL, std::string(what) + ": null data");
}

Mat ws_mat(Ctx& c, const std::string& key, int64_t rows, int64_t cols, int dtype) {
  Mat m;
  m.rows = rows;
  m.cols = cols;
  m.dtype = dtype;
  m.v.rows = rows;
  m.v.cols = cols;
  m.v.ld = round8(std::max<int64_t>(cols, 1));
  m.v.ps = round8(std::max<int64_t>(rows, 1) * m.v.ld);
  m.v.p = c.ws.get(key + (dtype == QPINV_F64 ? ":f64" : ":f32"), 4 * m.v.ps * esize(dtype));
  return m;
}

void gemm(Ctx& c, Prec p, const Mat& A, const Mat& B, const Epilogue& e, hipStream_t s, double* red) {
  if (A.cols != B.rows) throw Error(QPINV_EINVAL, "gemm: inner dimensions differ");
  const int64_t M = A.rows, N = B.cols, K = A.cols;
  if (p == P_F32 && c.split_f32 && bf16x3_fits(M, N, K)) p = P_BF16X3;
  const int cfg = c.config_for(p, M, N, K, s);
  const double f = 32.0 * (double)M * (double)N * (double)K;
  c.flops += f;
  if (!c.opt.gemm_timing || c.no_alloc) {
    qgemm(p, A.v, B.v, M, N, K, e, red, c.scratch, s, cfg);
    return;
  }
  if (c.events_used == c.events.size()) {
    hipEvent_t a, b;
    QP_HIP(hipEventCreate(&a));
    QP_HIP(hipEventCreate(&b));
    c.events.emplace_back(a, b);
    c.event_flops.push_back(0.0);
    c.event_key.push_back(0);
  }
  auto& ev = c.events[c.events_used];
  c.event_flops[c.events_used] = f;
  c.event_key[c.events_used] = (int)p * 64 + cfg;
  ++c.events_used;
  QP_HIP(hipEventRecord(ev.first, s));
  qgemm(p, A.v, B.v, M, N, K, e, red, c.scratch, s, cfg);
  QP_HIP(hipEventRecord(ev.second, s));
}

int gemm_stats(Ctx& c, double* out, int max_rows) {
  std::map<int, std::array<double, 3>> agg;  // key -> launches, flops, ms
  for (size_t i = 0; i < c.events_used; ++i) {
    QP_HIP(hipEventSynchronize(c.events[i].second));
    float t = 0.f;
    QP_HIP(hipEventElapsedTime(&t, c.events[i].first, c.events[i].second));
    auto& a = agg[c.event_key[i]];
    a[0] += 1.0;
    a[1] += c.event_flops[i];
    a[2] += t;
  }
  c.events_used = 0;
  int rows = 0;
  for (auto& kv : agg) {
    if (rows >= max_rows) break;
    double* r = out + 5 * rows;
    r[0] = kv.first / 64;
    r[1] = kv.first % 64;
    r[2] = kv.second[0];
    r[3] = kv.second[1];
    r[4] = kv.second[2];
    ++rows;
  }
  return rows;
}

void check_method(int method, int& order) {
  switch (method) {
    case QPINV_NS:
      if (order == 0) order = 2;
      if (order != 2) throw Error(QPINV_EINVAL, "Newton-Schulz has order 2");
      break;
    case QPINV_HPI:
      if (order < 2 || order > 64) throw Error(QPINV_EINVAL, "hyperpower order must be in [2, 64]");
      break;
    case QPINV_QSAI:
      if (order == 0) order = 10;
      if (order != 10) throw Error(QPINV_EINVAL, "QSAI has order 10");
      break;
    case QPINV_QHPI19:
      if (order == 0) order = 19;
      if (order != 19) throw Error(QPINV_EINVAL, "QHPI19 has order 19");
      break;
    case QPINV_QRAPID:
      if (order == -1) order = 5;
      if (order < 0 || order > 32) throw Error(QPINV_EINVAL, "QRAPID step parameter N must be in [0, 32]");
      break;
    default:
      throw Error(QPINV_EINVAL, "unknown method");
  }
}

// Local order p of a method (R_{j+1} ~ R_j^p): NS 2, hyperpower p, QSAI 10, QHPI19 19, and for
// QRAPID(N) nu_N = 11 a_{N-1} + 7 a_{N-2} + 1 with the Fibonacci numbers a (a_{-1} = 1, a_{-2} = -1).
static int convergence_order(int method, int order) {
  switch (method) {
    case QPINV_NS: return 2;
    case QPINV_HPI: return order;
    case QPINV_QSAI: return 10;
    case QPINV_QHPI19: return 19;
    default: {
      auto fib = [](int k) {
        long a = 0, b = 1;  // a_0, a_1
        if (k >= 0) {
          for (int i = 0; i < k; ++i) {
            const long t = a + b;
            a = b;
            b = t;
          }
          return a;
        }
        for (int i = 0; i < -k; ++i) {
          const long t = b - a;
          b = a;
          a = t;
        }
        return a;
      };
      return (int)(11 * fib(order - 1) + 7 * fib(order - 2) + 1);
    }
  }
}

// ------------------------------------------------------------------------------------------------
// one iteration
// ------------------------------------------------------------------------------------------------
void chain(Ctx& c, int method, int order, int side, Prec p, const Mat& A, const Mat& Xc, const Mat& Xn, double* red,
           hipStream_t s, Mat* Rout) {
  const int dt = store_of(p);
  const int64_t m = A.rows, n = A.cols;
  const bool left = side == QPINV_SIDE_LEFT;
  const int64_t sd = left ? n : m;
  auto sq = [&](int k) { return ws_mat(c, "sq" + std::to_string(k), sd, sd, dt); };
  auto xb = [&](int k) { return ws_mat(c, "xb" + std::to_string(k), n, m, dt); };
  // side product X A (left) or A X (right)
  auto prod = [&](const Epilogue& e) {
    if (left)
      gemm(c, p, Xc, A, e, s);
    else
      gemm(c, p, A, Xc, e, s);
  };
  // update: T X (left) or X T (right) into Xn, reducing against Xc
  auto apply = [&](const Mat& T) {
    Epilogue e = epi1(Xn);
    e.nin = 1;
    e.in[0] = Xc.v;
    e.b[0][0] = 0.0;
    e.ref = 0;
    e.reduce = red != nullptr;
    if (left)
      gemm(c, p, T, Xc, e, s, red);
    else
      gemm(c, p, Xc, T, e, s, red);
  };

  switch (method) {
    case QPINV_NS: {
      // T = 2I - (side product) = I + R; X+ = T X
      Mat T = sq(0);
      Epilogue e = epi1(T, -1.0, 2.0);
      Mat R;
      if (Rout) {
        R = sq(1);
        e.nout = 2;
        e.out[1] = R.v;
        e.a[1] = -1.0;
        e.g[1] = 1.0;
      }
      prod(e);
      if (Rout) *Rout = R;
      apply(T);
      break;
    }
    case QPINV_HPI: {
      // R = I - prod, S = I + R; S <- I + R S (p - 2 times); X+ = S X
      Mat R = sq(0), S0 = sq(1), S1 = sq(2);
      Epilogue e = epi1(R, -1.0, 1.0);
      e.nout = 2;
      e.out[1] = S0.v;
      e.a[1] = -1.0;
      e.g[1] = 2.0;
      prod(e);
      if (Rout) *Rout = R;
      Mat cur = S0, nxt = S1;
      for (int k = 0; k < order - 2; ++k) {
        gemm(c, p, R, cur, epi1(nxt, 1.0, 1.0), s);
        std::swap(cur, nxt);
      }
      apply(cur);
      break;
    }
    case QPINV_QSAI: {
      // Algorithm 2: R, R^2, R^4-level factors P1 = I + b1 R^2 + R^4, P2 = I + b2 R^2 + R^4,
      // Q = P1 P2, T = (I + R) Q, X+ = T X.
      Mat R = sq(0), Sp = sq(1), R2 = sq(2), P1 = sq(3), P2 = sq(4);
      Epilogue e = epi1(R, -1.0, 1.0);
      e.nout = 2;
      e.out[1] = Sp.v;
      e.a[1] = -1.0;
      e.g[1] = 2.0;
      prod(e);
      if (Rout) *Rout = R;
      gemm(c, p, R, R, epi1(R2), s);
      Epilogue e4;
      e4.nout = 2;
      e4.out[0] = P1.v;
      e4.out[1] = P2.v;
      e4.a[0] = e4.a[1] = 1.0;
      e4.nin = 1;
      e4.in[0] = R2.v;
      e4.b[0][0] = kBeta1;
      e4.b[1][0] = kBeta2;
      e4.g[0] = e4.g[1] = 1.0;
      gemm(c, p, R2, R2, e4, s);
      Mat Qm = Rout ? sq(5) : R;  // R is dead unless the caller wants it
      gemm(c, p, P1, P2, epi1(Qm), s);
      Mat T = R2;
      gemm(c, p, Sp, Qm, epi1(T), s);
      apply(T);
      break;
    }
    case QPINV_QHPI19: {
      // Algorithm 3: R, R^2, R^4; U = (I + d1 R^2 + R^4)(I + d2 R^2 + R^4); V = U + d3 R^2;
      // W = U + e1 R^2 + e2 R^4; Gamma = V W + c1 R^2 + c2 R^4; T = I + (R + R^2) Gamma; X+ = T X.
      Mat R = sq(0), R2 = sq(1), R4 = sq(2), S = sq(3), P1 = sq(4), P2 = sq(5), V = sq(6), W = sq(7);
      prod(epi1(R, -1.0, 1.0));
      if (Rout) *Rout = R;
      {  // R^2 and S = R + R^2
        Epilogue e = epi1(R2);
        e.nout = 2;
        e.out[1] = S.v;
        e.a[1] = 1.0;
        e.nin = 1;
        e.in[0] = R.v;
        e.b[1][0] = 1.0;
        gemm(c, p, R, R, e, s);
      }
      {  // R^4 and the two quadratic factors
        Epilogue e = epi1(R4);
        e.nout = 3;
        e.out[1] = P1.v;
        e.out[2] = P2.v;
        e.a[1] = e.a[2] = 1.0;
        e.nin = 1;
        e.in[0] = R2.v;
        e.b[1][0] = kD1;
        e.b[2][0] = kD2;
        e.g[1] = e.g[2] = 1.0;
        gemm(c, p, R2, R2, e, s);
      }
      {  // U = P1 P2 -> V, W
        Epilogue e;
        e.nout = 2;
        e.out[0] = V.v;
        e.out[1] = W.v;
        e.a[0] = e.a[1] = 1.0;
        e.nin = 2;
        e.in[0] = R2.v;
        e.in[1] = R4.v;
        e.b[0][0] = kD3;
        e.b[1][0] = kE1;
        e.b[1][1] = kE2;
        gemm(c, p, P1, P2, e, s);
      }
      Mat G = P1;  // P1, P2 are dead
      {
        Epilogue e = epi1(G);
        e.nin = 2;
        e.in[0] = R2.v;
        e.in[1] = R4.v;
        e.b[0][0] = kC1;
        e.b[0][1] = kC2;
        gemm(c, p, V, W, e, s);
      }
      Mat T = P2;
      gemm(c, p, S, G, epi1(T, 1.0, 1.0), s);
      apply(T);
      break;
    }
    case QPINV_QRAPID: {
      const int N = order;
      if (left) {
        // Q = X A; H1 = 7I - Q; H2 = 15I - Q H1; F = 13I - Q H2; U = F X / 4;
        // V = U + X - Q U; Z_l = W + Y - (Y A) W; X+ = Z + X - Q Z.
        Mat Q = sq(0), H1 = sq(1), H2 = sq(2), YA = sq(3);
        Mat B0 = xb(0), B1 = xb(1), B2 = xb(2);
        Epilogue e = epi1(Q);
        e.nout = Rout ? 3 : 2;
        e.out[1] = H1.v;
        e.a[1] = -1.0;
        e.g[1] = 7.0;
        Mat R;
        if (Rout) {
          R = sq(4);
          e.out[2] = R.v;
          e.a[2] = -1.0;
          e.g[2] = 1.0;
        }
        gemm(c, p, Xc, A, e, s);
        if (Rout) *Rout = R;
        gemm(c, p, Q, H1, epi1(H2, -1.0, 15.0), s);
        gemm(c, p, Q, H2, epi1(H1, -1.0, 13.0), s);  // F into H1
        gemm(c, p, H1, Xc, epi1(B0, 0.25), s);       // U
        {
          Epilogue ev = epi1(B1, -1.0);
          ev.nin = 2;
          ev.in[0] = B0.v;
          ev.in[1] = Xc.v;
          ev.b[0][0] = 1.0;
          ev.b[0][1] = 1.0;
          gemm(c, p, Q, B0, ev, s);  // V
        }
        Mat Y = B0, W = B1, Z = B1, F = B2;
        for (int l = 0; l < N; ++l) {
          gemm(c, p, Y, A, epi1(YA), s);
          Epilogue ez = epi1(F, -1.0);
          ez.nin = 2;
          ez.in[0] = W.v;
          ez.in[1] = Y.v;
          ez.b[0][0] = 1.0;
          ez.b[0][1] = 1.0;
          gemm(c, p, YA, W, ez, s);
          Z = F;
          Mat freed = Y;
          Y = W;
          W = Z;
          F = freed;
        }
        Epilogue ex = epi1(Xn, -1.0);
        ex.nin = 2;
        ex.in[0] = Z.v;
        ex.in[1] = Xc.v;
        ex.b[0][0] = 1.0;
        ex.b[0][1] = 1.0;
        ex.ref = 1;
        ex.reduce = red != nullptr;
        gemm(c, p, Q, Z, ex, s, red);
      } else {
        // P = A X; H1 = 7I - P; H2 = 15I - P H1; F = 13I - P H2; U = X F / 4;
        // V = U + X (I - A U); Z_l = W + Y (I - A W); X+ = Z + X (I - A Z).
        Mat P = sq(0), H1 = sq(1), H2 = sq(2), E = sq(3);
        Mat B0 = xb(0), B1 = xb(1), B2 = xb(2);
        Epilogue e = epi1(P);
        e.nout = Rout ? 3 : 2;
        e.out[1] = H1.v;
        e.a[1] = -1.0;
        e.g[1] = 7.0;
        Mat R;
        if (Rout) {
          R = sq(4);
          e.out[2] = R.v;
          e.a[2] = -1.0;
          e.g[2] = 1.0;
        }
        gemm(c, p, A, Xc, e, s);
        if (Rout) *Rout = R;
        gemm(c, p, P, H1, epi1(H2, -1.0, 15.0), s);
        gemm(c, p, P, H2, epi1(H1, -1.0, 13.0), s);  // F into H1
        gemm(c, p, Xc, H1, epi1(B0, 0.25), s);       // U
        gemm(c, p, A, B0, epi1(E, -1.0, 1.0), s);     // I - A U
        {
          Epilogue ev = epi1(B1);
          ev.nin = 1;
          ev.in[0] = B0.v;
          ev.b[0][0] = 1.0;
          gemm(c, p, Xc, E, ev, s);  // V
        }
        Mat Y = B0, W = B1, Z = B1, F = B2;
        for (int l = 0; l < N; ++l) {
          gemm(c, p, A, W, epi1(E, -1.0, 1.0), s);
          Epilogue ez = epi1(F);
          ez.nin = 1;
          ez.in[0] = W.v;
          ez.b[0][0] = 1.0;
          gemm(c, p, Y, E, ez, s);
          Z = F;
          Mat freed = Y;
          Y = W;
          W = Z;
          F = freed;
        }
        gemm(c, p, A, Z, epi1(E, -1.0, 1.0), s);
        Epilogue ex = epi1(Xn);
        ex.nin = 2;
        ex.in[0] = Z.v;
        ex.in[1] = Xc.v;
        ex.b[0][0] = 1.0;
        ex.b[0][1] = 0.0;
        ex.ref = 1;
        ex.reduce = red != nullptr;
        gemm(c, p, Xc, E, ex, s, red);
      }
      break;
    }
    default:
      throw Error(QPINV_EINVAL, "unknown method");
  }
}

// ------------------------------------------------------------------------------------------------
// helpers of the solve
// ------------------------------------------------------------------------------------------------
namespace {

void to_host(Ctx& c, const double* dev, int count, hipStream_t s) {
  QP_HIP(hipMemcpyAsync(c.hsc, dev, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  QP_HIP(hipStreamSynchronize(s));
}

void convert_mat(const Mat& src, const Mat& dst, hipStream_t s) {
  if (src.rows != dst.rows || src.cols != dst.cols) throw Error(QPINV_EINVAL, "convert: shape mismatch");
  if (src.dtype == QPINV_F32 && dst.dtype == QPINV_F32)
    convert<float, float>(src.v, dst.v, src.rows, src.cols, s);
  else if (src.dtype == QPINV_F32)
    convert<float, double>(src.v, dst.v, src.rows, src.cols, s);
  else if (dst.dtype == QPINV_F32)
    convert<double, float>(src.v, dst.v, src.rows, src.cols, s);
  else
    convert<double, double>(src.v, dst.v, src.rows, src.cols, s);
}

// One update of the FP64 finish evaluated in mixed precision (NS, HPI, QSAI, QHPI19: X+ = T(R) X with
// T = I + T'): the residual R = I - X A (left) or I - A X (right) is an FP64 product of the FP64
// iterate, and X+ = X + T' X is summed in FP64; T' (a polynomial in R without the identity term) and
// the correction T' X are FP32 products.  Near convergence R and T' are small, so the FP32 rounding of
// the correction is relative to |T' X|, far below |X| u_64-level effects of the FP64 residual.
void chain_refined(Ctx& c, int method, int order, int side, const Mat& A64, const Mat& Xc, const Mat& Xn,
                   double* red, hipStream_t s) {
  const int64_t m = A64.rows, n = A64.cols;
  const bool left = side == QPINV_SIDE_LEFT;
  const int64_t sd = left ? n : m;
  auto sq = [&](int k) { return ws_mat(c, "rf" + std::to_string(k), sd, sd, QPINV_F32); };
  Mat R64 = ws_mat(c, "rfR64", sd, sd, QPINV_F64), S64 = ws_mat(c, "rfS64", sd, sd, QPINV_F64);
  {  // R = I - prod and (for HPI) S = I + R = 2I - prod, in FP64
    Epilogue e = epi1(R64, -1.0, 1.0);
    if (method == QPINV_HPI) {
      e.nout = 2;
      e.out[1] = S64.v;
      e.a[1] = -1.0;
      e.g[1] = 2.0;
    }
    if (left)
      gemm(c, P_F64, Xc, A64, e, s);
    else
      gemm(c, P_F64, A64, Xc, e, s);
  }
  Mat R = sq(0);
  convert_mat(R64, R, s);
  Mat X32 = ws_mat(c, "rfX", n, m, QPINV_F32);
  convert_mat(Xc, X32, s);
  Mat Tp;  // T - I
  switch (method) {
    case QPINV_NS:  // T = I + R
      Tp = R;
      break;
    case QPINV_HPI: {  // S = I + R; S <- I + R S (p - 3 times); T - I = R S
      Mat cur = sq(1), nxt = sq(2);
      convert_mat(S64, cur, s);
      if (order == 2) {
        Tp = R;
        break;
      }
      for (int k = 0; k < order - 3; ++k) {
        gemm(c, P_F32, R, cur, epi1(nxt, 1.0, 1.0), s);
        std::swap(cur, nxt);
      }
      Tp = nxt;
      gemm(c, P_F32, R, cur, epi1(Tp), s);
      break;
    }
    case QPINV_QSAI: {
      // P1 = I + a, P2 = I + b with a = b1 R^2 + R^4, b = b2 R^2 + R^4; Q = P1 P2 = I + Q',
      // Q' = a b + a + b; T = (I + R) Q, T - I = R Q' + R + Q'
      Mat R2 = sq(1), Pa = sq(2), Pb = sq(3), Qp = sq(4);
      Tp = sq(5);
      gemm(c, P_F32, R, R, epi1(R2), s);
      Epilogue e4;
      e4.nout = 2;
      e4.out[0] = Pa.v;
      e4.out[1] = Pb.v;
      e4.a[0] = e4.a[1] = 1.0;
      e4.nin = 1;
      e4.in[0] = R2.v;
      e4.b[0][0] = kBeta1;
      e4.b[1][0] = kBeta2;
      gemm(c, P_F32, R2, R2, e4, s);
      Epilogue eq = epi1(Qp);
      eq.nin = 2;
      eq.in[0] = Pa.v;
      eq.in[1] = Pb.v;
      eq.b[0][0] = 1.0;
      eq.b[0][1] = 1.0;
      gemm(c, P_F32, Pa, Pb, eq, s);
      Epilogue et = epi1(Tp);
      et.nin = 2;
      et.in[0] = R.v;
      et.in[1] = Qp.v;
      et.b[0][0] = 1.0;
      et.b[0][1] = 1.0;
      gemm(c, P_F32, R, Qp, et, s);
      break;
    }
    default: {  // QHPI19: the chain of Algorithm 3 from R; T - I = (R + R^2) Gamma
      Mat R2 = sq(1), R4 = sq(2), Sm = sq(3), P1 = sq(4), P2 = sq(5), V = sq(6), W = sq(7);
      {
        Epilogue e = epi1(R2);
        e.nout = 2;
        e.out[1] = Sm.v;
        e.a[1] = 1.0;
        e.nin = 1;
        e.in[0] = R.v;
        e.b[1][0] = 1.0;
        gemm(c, P_F32, R, R, e, s);
      }
      {
        Epilogue e = epi1(R4);
        e.nout = 3;
        e.out[1] = P1.v;
        e.out[2] = P2.v;
        e.a[1] = e.a[2] = 1.0;
        e.nin = 1;
        e.in[0] = R2.v;
        e.b[1][0] = kD1;
        e.b[2][0] = kD2;
        e.g[1] = e.g[2] = 1.0;
        gemm(c, P_F32, R2, R2, e, s);
      }
      {
        Epilogue e;
        e.nout = 2;
        e.out[0] = V.v;
        e.out[1] = W.v;
        e.a[0] = e.a[1] = 1.0;
        e.nin = 2;
        e.in[0] = R2.v;
        e.in[1] = R4.v;
        e.b[0][0] = kD3;
        e.b[1][0] = kE1;
        e.b[1][1] = kE2;
        gemm(c, P_F32, P1, P2, e, s);
      }
      Mat G = P1;
      {
        Epilogue e = epi1(G);
        e.nin = 2;
        e.in[0] = R2.v;
        e.in[1] = R4.v;
        e.b[0][0] = kC1;
        e.b[0][1] = kC2;
        gemm(c, P_F32, V, W, e, s);
      }
      Tp = P2;
      gemm(c, P_F32, Sm, G, epi1(Tp), s);
      break;
    }
  }
  Mat D = ws_mat(c, "rfD", n, m, QPINV_F32);
  if (left)
    gemm(c, P_F32, Tp, X32, epi1(D), s);
  else
    gemm(c, P_F32, X32, Tp, epi1(D), s);
  if (add_delta_blocks(n, m) * 2 > c.scratch.capacity) throw Error(QPINV_EINVAL, "refined finish: scratch too small");
  add_delta(Xc.v, D.v, Xn.v, n, m, red, c.scratch.partial, s);
}


void x0_into(const Mat& A, double alpha, const Mat& X, hipStream_t s) {
  if (A.dtype == QPINV_F32 && X.dtype == QPINV_F32)
    x0_scaled_adjoint<float, float>(A.v, A.rows, A.cols, alpha, X.v, s);
  else if (A.dtype == QPINV_F32)
    x0_scaled_adjoint<float, double>(A.v, A.rows, A.cols, alpha, X.v, s);
  else if (X.dtype == QPINV_F32)
    x0_scaled_adjoint<double, float>(A.v, A.rows, A.cols, alpha, X.v, s);
  else
    x0_scaled_adjoint<double, double>(A.v, A.rows, A.cols, alpha, X.v, s);
}

// norms of a matrix into host h[0..3] = {||M||_F^2, ||M||_1, ||M||_inf, nonfinite count}
void norms_host(Ctx& c, const Mat& M, double h[4], hipStream_t s) {
  double* work = static_cast<double*>(c.ws.get("normwork", sizeof(double) * norms_work_doubles(M.rows, M.cols)));
  if (M.dtype == QPINV_F32)
    norms<float>(M.v, M.rows, M.cols, c.dsc + 8, work, s);
  else
    norms<double>(M.v, M.rows, M.cols, c.dsc + 8, work, s);
  to_host(c, c.dsc + 8, 4, s);
  std::memcpy(h, c.hsc, sizeof(double) * 4);
}

double power_host(Ctx& c, const Mat& M, int steps, hipStream_t s, double* prev = nullptr) {
  double* work = static_cast<double*>(c.ws.get("powwork", sizeof(double) * power_work_doubles(M.rows, M.cols)));
  if (M.dtype == QPINV_F32)
    power_sigma1_sq<float>(M.v, M.rows, M.cols, steps, c.opt.power_seed, c.dsc + 16, work, s);
  else
    power_sigma1_sq<double>(M.v, M.rows, M.cols, steps, c.opt.power_seed, c.dsc + 16, work, s);
  to_host(c, c.dsc + 16, 2, s);
  if (prev) *prev = c.hsc[1];
  return c.hsc[0];
}

// ||X A X - X||_F^2 in FP64 (A64, X64 double storage)
double e2_sq(Ctx& c, const Mat& A64, const Mat& X64, hipStream_t s) {
  const int64_t m = A64.rows, n = A64.cols;
  Mat XA = ws_mat(c, "e2_xa", n, n, QPINV_F64);
  Mat O = ws_mat(c, "e2_out", n, m, QPINV_F64);
  gemm(c, P_F64, X64, A64, epi1(XA), s);
  Epilogue e = epi1(O);
  e.nin = 1;
  e.in[0] = X64.v;
  e.ref = 0;
  e.reduce = true;
  gemm(c, P_F64, XA, X64, e, s, c.dsc + 24);
  to_host(c, c.dsc + 24, 2, s);
  return c.hsc[0];
}

// ||X A X - X||_F^2 from the residual of X: R = I - X A (left, n x n) gives X A X - X = -R X,
// R = I - A X (right, m x m) gives -X R.  Computed in the precision p of the stored R and X.
double e2_sq_from_residual(Ctx& c, Prec p, int side, const Mat& R, const Mat& X, hipStream_t s) {
  Mat O = ws_mat(c, "e2r_out", X.rows, X.cols, X.dtype);
  Epilogue e = epi1(O);
  e.reduce = true;
  if (side == QPINV_SIDE_LEFT)
    gemm(c, p, R, X, e, s, c.dsc + 28);
  else
    gemm(c, p, X, R, e, s, c.dsc + 28);
  to_host(c, c.dsc + 28, 2, s);
  return c.hsc[0];
}

// ||A X A - A||_F^2 in the precision p (A and X of p's storage)
double e1_sq(Ctx& c, Prec p, const Mat& A, const Mat& X, hipStream_t s) {
  const int64_t m = A.rows, n = A.cols;
  const int dt = store_of(p);
  Mat O = ws_mat(c, "e1_out", m, n, dt);
  Epilogue e = epi1(O);
  e.nin = 1;
  e.in[0] = A.v;
  e.ref = 0;
  e.reduce = true;
  if (m >= n) {
    Mat XA = ws_mat(c, "e1_xa", n, n, dt);
    gemm(c, p, X, A, epi1(XA), s);
    gemm(c, p, A, XA, e, s, c.dsc + 26);
  } else {
    Mat AX = ws_mat(c, "e1_ax", m, m, dt);
    gemm(c, p, A, X, epi1(AX), s);
    gemm(c, p, AX, A, e, s, c.dsc + 26);
  }
  to_host(c, c.dsc + 26, 2, s);
  return c.hsc[0];
}

// Projection of an FP64 iterate X (n x m) toward A^dagger with the Penrose conditions (Section 2), into O.
//   mode 1: O = X A X (condition (b); a fixed point of every {2}-inverse of A).
//   mode 2: O = (X A)^H X (A X)^H, which equals X for A^dagger by conditions (b)-(d).  Its rows lie in
//           range(A^H) and its columns in range(A), the invariants every exact iterate keeps (Proposition 3.1):
//           it removes what rounding put outside them.  Near-null directions of a numerically rank-deficient
//           A take rounding that the update multiplies by its order, and the blocks of X that map them to
//           range directions are fixed points of the update and of X A X; this projection removes both.
void penrose_project(Ctx& c, int mode, const Mat& A64, const Mat& X64, const Mat& O, hipStream_t s) {
  const int64_t m = A64.rows, n = A64.cols;
  Mat XA = ws_mat(c, "pf_xa", n, n, QPINV_F64);
  gemm(c, P_F64, X64, A64, epi1(XA), s);
  if (mode == 1) {
    gemm(c, P_F64, XA, X64, epi1(O), s);
    return;
  }
  Mat AX = ws_mat(c, "pf_ax", m, m, QPINV_F64);
  gemm(c, P_F64, A64, X64, epi1(AX), s);
  Mat H1 = ws_mat(c, "pf_h1", n, n, QPINV_F64), H2 = ws_mat(c, "pf_h2", m, m, QPINV_F64);
  Mat P1 = ws_mat(c, "pf_p1", n, m, QPINV_F64);
  x0_into(XA, 1.0, H1, s);
  x0_into(AX, 1.0, H2, s);
  gemm(c, P_F64, H1, X64, epi1(P1), s);
  gemm(c, P_F64, P1, H2, epi1(O), s);
}

struct IterSet {
  Mat b[4];
};

}  // namespace

// ------------------------------------------------------------------------------------------------
// the solve
// ------------------------------------------------------------------------------------------------
int solve(Ctx& c, int method, int order, const qpinv_qmat* Aq, int scaling, double am, double tol, int max_iter,
          int stop, int precision, qpinv_qmat* Xq, qpinv_info* info, hipStream_t s) {
  const double t0 = now_s();
  check_method(method, order);
  validate(Aq, "A");
  validate(Xq, "X");
  if (Xq->rows != Aq->cols || Xq->cols != Aq->rows) throw Error(QPINV_EINVAL, "X must be n x m for A m x n");
  if (!(tol >= 0.0) || max_iter < 1) throw Error(QPINV_EINVAL, "tol must be >= 0 and max_iter >= 1");
  if (stop < STOP_DX_ABS || stop > STOP_GUARDED) throw Error(QPINV_EINVAL, "bad stop rule");
  if (precision < QPINV_PREC_F64 || precision > QPINV_PREC_MIXED) throw Error(QPINV_EINVAL, "bad precision");
  if (scaling < QPINV_ALPHA_POWER || scaling > QPINV_X0_GIVEN) throw Error(QPINV_EINVAL, "bad scaling");
  if (scaling == QPINV_ALPHA_GIVEN && !(am > 0.0)) throw Error(QPINV_EINVAL, "ALPHA_GIVEN needs alpha > 0");
  if (c.opt.penrose_finish == 2 && precision == QPINV_PREC_F32)
    throw Error(QPINV_EINVAL, "penrose_finish = 2 needs FP64 updates (precision F64, F32_F64FINISH or MIXED)");

  qpinv_info inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.e1_rel = -1.0;
  const double flops0 = c.flops;
  const Mat A0 = from_abi(*Aq);
  const Mat Xout = from_abi(*Xq);
  const int64_t m = A0.rows, n = A0.cols;
  int side = c.opt.side;
  if (side == QPINV_SIDE_AUTO) side = (m > n) ? QPINV_SIDE_LEFT : QPINV_SIDE_RIGHT;
  inf.side = side;
  auto finish = [&](int status) {
    inf.seconds = now_s() - t0;
    inf.gemm_flops = c.flops - flops0;
    if (info) *info = inf;
    return status;
  };
  if (m == 0 || n == 0) return finish(QPINV_OK);
  if (small_eligible(c, method, order, scaling, stop, precision, m, n))
    return finish(small_solve(c, method, order, A0, scaling, am, tol, max_iter, stop, precision, Xout, inf, s));
  // the ladder's FP32-storage products (its FP32 phase and the finish's corrections) as three BF16 products;
  // not in an allocation-free call, whose stage buffer may not grow (the split copies need one)
  struct SplitScope {
    Ctx& c;
    SplitScope(Ctx& cx, bool on) : c(cx) { c.split_f32 = on; }
    ~SplitScope() { c.split_f32 = false; }
  } split_scope(c, precision == QPINV_PREC_MIXED && c.opt.mixed_split != 0 && !c.no_alloc);

  // A in each storage type on demand
  Mat Acache[2];
  bool have[2] = {false, false};
  auto A_of = [&](int dt) -> Mat {
    const int k = dt == QPINV_F64 ? 1 : 0;
    if (A0.dtype == dt) return A0;
    if (!have[k]) {
      Acache[k] = ws_mat(c, "A", m, n, dt);
      convert_mat(A0, Acache[k], s);
      have[k] = true;
    }
    return Acache[k];
  };

  double nh[4];
  norms_host(c, A0, nh, s);
  if (nh[3] > 0) return finish(QPINV_ENONFINITE);
  const double normA = std::sqrt(nh[0]);
  if (normA == 0.0) {  // A = 0: the pseudoinverse is 0
    Mat Xz = ws_mat(c, "zero", n, m, Xout.dtype);
    zero_doubles(static_cast<double*>(Xz.v.p), 4 * Xz.v.ps * (int64_t)esize(Xz.dtype) / 8, s);
    convert_mat(Xz, Xout, s);
    QP_HIP(hipStreamSynchronize(s));
    return finish(QPINV_OK);
  }

  // precision phases
  std::vector<Prec> phases;
  switch (precision) {
    case QPINV_PREC_F64: phases = {P_F64}; break;
    case QPINV_PREC_F32: phases = {P_F32}; break;
    case QPINV_PREC_F32_F64FINISH: phases = {P_F32, P_F64}; break;
    default: phases = {P_BF16, P_F32, P_F64}; break;
  }
  const bool has_finish = phases.size() > 1 && phases.back() == P_F64;
  size_t ph = 0;

  // scaling
  double alpha = 0.0;
  double alpha_classical = 0.0;
  bool learned = false;
  if (scaling == QPINV_ALPHA_POWER || scaling == QPINV_ALPHA_LEARNED) {
    double prev = 0.0;
    inf.sigma1_sq_est = power_host(c, A0, c.opt.power_steps, s, &prev);
    double mu = am > 0.0 ? am : 1.0;
    alpha_classical = 1.0 / inf.sigma1_sq_est;
    if (scaling == QPINV_ALPHA_LEARNED) {
      if (!mlp_ready(c)) {
        inf.fallback_used = 1;  // no network loaded: the classical alpha
      } else {
        // network input row (s1sq, s1sq_prev, fro, norm1, norminf, m, n) -> mu
        double* raw = c.dsc + 48;
        double* hraw = c.hsc + 48;
        const double row[7] = {inf.sigma1_sq_est, prev, normA, nh[1], nh[2], (double)m, (double)n};
        std::memcpy(hraw, row, sizeof(row));
        QP_HIP(hipMemcpyAsync(raw, hraw, sizeof(row), hipMemcpyHostToDevice, s));
        mlp_predict(c, raw, 1, c.dsc + 56, s);
        to_host(c, c.dsc + 56, 1, s);
        double mul = c.hsc[0];
        // clamp: sigma_1 <= U = min(||A||_F, sqrt(||A||_1 ||A||_inf)) makes mu >= s1sq / U^2 a certified
        // lower end (alpha >= 1/U^2 > 0); the upper end 1.9 is not certified (sigma1_est^2 underestimates
        // sigma_1^2), which the residual guard and the restart on divergence or max_iter cover
        const double U2 = std::min(nh[0], nh[1] * nh[2]);
        const double lo = inf.sigma1_sq_est / U2, hi = 1.9;
        if (!std::isfinite(mul) || mul < lo || mul > hi) {
          inf.alpha_clamped = 1;
          mul = std::isfinite(mul) ? std::min(std::max(mul, lo), hi) : 1.0;
        }
        mu = mul;
        learned = true;
      }
    }
    alpha = mu / inf.sigma1_sq_est;
    inf.mu_used = mu;
  } else if (scaling == QPINV_ALPHA_FROB) {
    alpha = 1.0 / nh[0];
  } else if (scaling == QPINV_ALPHA_GIVEN) {
    alpha = am;
  }
  inf.alpha_used = alpha;

  // iterate buffers per storage type
  IterSet sets[2];
  bool have_set[2] = {false, false};
  auto set_of = [&](int dt) -> IterSet& {
    const int k = dt == QPINV_F64 ? 1 : 0;
    if (!have_set[k])
      for (int i = 0; i < 4; ++i) sets[k].b[i] = ws_mat(c, "X" + std::to_string(i), n, m, dt);
    have_set[k] = true;
    return sets[k];
  };

  int dt = store_of(phases[0]);
  IterSet* S = &set_of(dt);
  int cur = 0;
  if (scaling == QPINV_X0_GIVEN) {
    double xh[4];
    norms_host(c, Xout, xh, s);
    if (xh[3] > 0) return finish(QPINV_ENONFINITE);
    convert_mat(Xout, S->b[cur], s);
  } else {
    x0_into(A_of(dt), alpha, S->b[cur], s);
  }

  StopController ctl(stop, tol);
  const int p_order = convergence_order(method, order);
  // FP64 finish updates: by default Newton-Schulz, the order-2 member of the family.  The finish starts
  // from an iterate at the FP32 floor, where squaring the error reaches the FP64 tolerance in one or
  // two updates of 2 products each, fewer products than one update of a higher order.
  int fin_method = c.opt.finish_method >= 0 ? c.opt.finish_method : method;
  int fin_order = c.opt.finish_method >= 0 ? 0 : order;
  check_method(fin_method, fin_order);
  const int p_finish = convergence_order(fin_method, fin_order);
  const double kF32Floor = 1e-6;  // relative error FP32 iterates cannot improve on
  std::vector<double> xnorm_hist(1, 0.0);  // ||X_j||_F by j (X_0 unknown = 0)
  int best_pair[2] = {-1, -1};             // buffer indices of X_{j*-1}, X_{j*}
  int best_j = -1;
  double* red = c.dsc;  // [0..1]
  int status = QPINV_OK;
  int returned_buf = cur;
  int returned_j = 0;
  bool done = false;
  double rprev = -1.0;
  int j = 0;
  double d_prev_finish = -1.0;

  Mat rsave[2];
  int rsave_j[2] = {-1, -1};  // index k of the iterate X_k whose residual R_k sits in each slot
  auto pick_free = [&](int a, int b, int cc) {
    for (int i = 0; i < 4; ++i)
      if (i != a && i != b && i != cc) return i;
    return -1;
  };

  // the learned alpha failed (divergence, no convergence within max_iter, or an estimated ||R_0||_2 above 1):
  // start over from the classical alpha
  auto restart_classical = [&]() {
    learned = false;
    inf.fallback_used = 1;
    alpha = alpha_classical;
    inf.alpha_used = alpha;
    inf.mu_used = 1.0;
    dt = store_of(phases[0]);
    ph = 0;
    S = &set_of(dt);
    cur = 0;
    x0_into(A_of(dt), alpha, S->b[cur], s);
    j = 0;
    inf.iters_bf16 = inf.iters_f32 = inf.iters_f64 = 0;
    ctl = StopController(stop, tol);
    xnorm_hist.assign(1, 0.0);
    best_pair[0] = best_pair[1] = -1;
    best_j = -1;
    rsave_j[0] = rsave_j[1] = -1;
    rprev = -1.0;
    d_prev_finish = -1.0;
  };

  while (!done) {
    const Prec p = phases[ph];
    if (j >= max_iter && learned) {
      restart_classical();
      continue;
    }
    if (j >= max_iter) {
      status = QPINV_ENOTCONVERGED;
      inf.stop_reason = QPINV_REASON_MAX_ITER;
      returned_buf = cur;
      returned_j = j;
      break;
    }
    const int nxt = pick_free(best_pair[0], best_pair[1], cur);
    const Mat Adt = A_of(store_of(p));
    Mat R;
    const bool main_phase = p != P_BF16 && !(has_finish && ph == phases.size() - 1);
    const bool keep_R = main_phase && stop == STOP_GUARDED;
    // the classical alpha (mu = 1) carries no more risk than the default; only a larger learned mu is checked,
    // and not under the E1 stop rule: ||A X A - A||_F <= tol ||A||_F certifies the result whatever alpha it
    // started from, and an inadmissible alpha never gets there (divergence or max_iter restart it)
    const bool guard_R = learned && j == 0 && inf.mu_used > 1.0 && stop != STOP_E1_REL;
    const bool want_R = (p == P_BF16) || keep_R || guard_R;
    const bool in_finish = has_finish && ph == phases.size() - 1;
    const int it_method = in_finish ? fin_method : method, it_order = in_finish ? fin_order : order;
    const bool refined = in_finish && c.opt.f64_refined && it_method != QPINV_QRAPID;
    if (refined)
      chain_refined(c, it_method, it_order, side, Adt, S->b[cur], S->b[nxt], red, s);
    else
      chain(c, it_method, it_order, side, p, Adt, S->b[cur], S->b[nxt], red, s, want_R ? &R : nullptr);
    if (guard_R) {
      // Theorem 1: alpha is admissible iff every |1 - alpha sigma_i^2| < 1; R_0 = I - X_0 A (or I - A X_0)
      // has exactly these eigenvalues (and 1 on the null space), so ||R_0||_2 > 1 means divergence
      const double r0 = std::sqrt(std::max(0.0, power_host(c, R, 3, s)));
      if (r0 > 1.0 + 1e-3) {
        restart_classical();
        continue;
      }
    }
    if (keep_R) {
      // keep R_{j} = residual of the iterate X_j this update started from (slot j % 2)
      const int slot = j % 2;
      rsave[slot] = ws_mat(c, "Rsave" + std::to_string(slot), R.rows, R.cols, R.dtype);
      QP_HIP(hipMemcpyAsync(rsave[slot].v.p, R.v.p, 4 * R.v.ps * esize(R.dtype), hipMemcpyDeviceToDevice, s));
      rsave_j[slot] = j;
    }
    double rnorm = -1.0;  // ||R_j||_2 estimate: only the BF16 phase's switch rule uses it
    if (p == P_BF16) rnorm = std::sqrt(std::max(0.0, power_host(c, R, c.opt.mixed_rnorm_steps, s)));
    to_host(c, red, 2, s);
    const double d_abs = std::sqrt(std::max(0.0, c.hsc[0]));
    const double xn = std::sqrt(std::max(0.0, c.hsc[1]));
    ++j;
    xnorm_hist.push_back(xn);
    if (p == P_BF16)
      ++inf.iters_bf16;
    else if (p == P_F32)
      ++inf.iters_f32;
    else
      ++inf.iters_f64;
    inf.final_dx_rel = xn > 0 ? d_abs / xn : 0.0;
    if (c.opt.verbose)
      fprintf(stderr, "[qpinv] it %d prec %d d_abs %.3e x %.3e d_rel %.3e rnorm %.3e\n", j, (int)p, d_abs, xn,
              inf.final_dx_rel, rnorm);

    const bool diverged = !std::isfinite(d_abs) || !std::isfinite(xn) || xn * normA > 1e20;
    if (diverged && learned) {
      restart_classical();
      continue;
    }
    if (diverged) {
      status = QPINV_EDIVERGED;
      inf.stop_reason = QPINV_REASON_DIVERGED;
      returned_buf = std::isfinite(xn) ? nxt : cur;
      returned_j = std::isfinite(xn) ? j : j - 1;
      break;
    }

    // ---------------------------------------------------------------- BF16 phase: switch rule
    if (p == P_BF16) {
      // next residual ~ ||R||^order; leave BF16 when that is below the switch threshold
      // or BF16 no longer reduces ||R|| (stagnation), or after max_bf16_iters
      const double pred = std::pow(rnorm, (double)std::max(order, 2));
      bool leave = rnorm < c.opt.mixed_switch || pred < c.opt.mixed_switch || inf.iters_bf16 >= c.opt.max_bf16_iters;
      if (rprev >= 0.0 && rnorm < 0.9 && rnorm > 0.5 * rprev) leave = true;
      if (rprev >= 0.0 && rnorm >= rprev - 1e-7) leave = true;
      rprev = rnorm;
      cur = nxt;
      if (leave) {
        ++ph;
        if (store_of(phases[ph]) != dt) {
          dt = store_of(phases[ph]);
          IterSet* S2 = &set_of(dt);
          convert_mat(S->b[cur], S2->b[0], s);
          S = S2;
          cur = 0;
        }
      }
      continue;
    }

    // ---------------------------------------------------------------- FP64 finish phase
    if (has_finish && ph == phases.size() - 1) {
      const double d = xn > 0 ? d_abs / xn : 0.0;
      const int fin_it = inf.iters_f64;
      if (c.opt.penrose_finish == 2) {
        // fixed schedule: the projection comes before the last update, which removes the first-order error
        // the projection leaves in the range directions; the updates before it converge the iterate (the
        // projection cubes whatever is not yet converged)
        const int total = std::max(2, c.opt.f64_finish_iters);
        if (fin_it >= total) {
          inf.stop_reason = QPINV_REASON_TOL;
          returned_buf = nxt;
          returned_j = j;
          done = true;
        } else if (fin_it == total - 1) {
          Mat O = ws_mat(c, "pf_out", n, m, QPINV_F64);
          penrose_project(c, 2, A_of(QPINV_F64), S->b[nxt], O, s);
          convert_mat(O, S->b[nxt], s);
        }
        d_prev_finish = d;
        cur = nxt;
        continue;
      }
      // in the asymptotic regime the next change is about d^p: once that is below tol the FP64 iterate
      // just computed is converged and a confirming step is not needed.  Not for order 2: the error of a
      // Newton-Schulz update is E A E, whose relative size carries a condition-number factor that d^2
      // does not, so that finish stops on its measured change
      const bool predicted = p_finish >= 3 && d <= 0.5 && std::pow(d, (double)p_finish) <= tol;
      if (d <= tol || predicted) {
        inf.stop_reason = QPINV_REASON_TOL;
        returned_buf = nxt;
        returned_j = j;
        done = true;
      } else if (d_prev_finish >= 0.0 && d > d_prev_finish) {
        inf.stop_reason = QPINV_REASON_RISE;
        returned_buf = cur;
        returned_j = j - 1;
        done = true;
      } else if (fin_it >= c.opt.f64_finish_iters) {
        inf.stop_reason = QPINV_REASON_TOL;
        returned_buf = nxt;
        returned_j = j;
        done = true;
      }
      d_prev_finish = d;
      cur = nxt;
      continue;
    }

    // ---------------------------------------------------------------- main phase: controller
    double e1r = -1.0;
    if (stop == STOP_E1_REL) {
      e1r = std::sqrt(std::max(0.0, e1_sq(c, p, Adt, S->b[nxt], s))) / normA;
      inf.e1_rel = e1r;
    }
    int dec = ctl.update(j, d_abs, xn, e1r);
    int chosen_buf = -1, chosen_j = -1, reason = -1;
    if (has_finish && (dec == D_CONTINUE || dec == D_NEWMIN)) {
      // leave the FP32 phase once X_j sits at the FP32 floor: its error is about d^p (asymptotic regime)
      const double d = xn > 0 ? d_abs / xn : 0.0;
      if (d <= 0.5 && std::pow(d, (double)p_order) <= kF32Floor) dec = D_TOL;
    }
    if (dec == D_DIVERGED) {
      status = QPINV_EDIVERGED;
      inf.stop_reason = QPINV_REASON_DIVERGED;
      returned_buf = cur;
      returned_j = j - 1;
      break;
    } else if (dec == D_TOL) {
      chosen_buf = nxt;
      chosen_j = j;
      reason = QPINV_REASON_TOL;
    } else if (dec == D_RISE) {
      // choose between X_{j*-1} and X_{j*} by ||XAX - X||_F / ||X||_F in FP64
      reason = QPINV_REASON_RISE;
      double ea, eb;
      const int ka = best_j - 1, kb = best_j;
      if (rsave_j[ka % 2] == ka && rsave_j[kb % 2] == kb) {
        // X A X - X = -R X (left) or -X R (right) with the residuals the chain already formed
        ea = std::sqrt(e2_sq_from_residual(c, p, side, rsave[ka % 2], S->b[best_pair[0]], s)) /
             std::max(xnorm_hist[ka], 1e-300);
        eb = std::sqrt(e2_sq_from_residual(c, p, side, rsave[kb % 2], S->b[best_pair[1]], s)) /
             std::max(xnorm_hist[kb], 1e-300);
      } else {
        const Mat A64 = A_of(QPINV_F64);
        Mat Xa64 = ws_mat(c, "cand", n, m, QPINV_F64);
        convert_mat(S->b[best_pair[0]], Xa64, s);
        ea = std::sqrt(e2_sq(c, A64, Xa64, s)) / std::max(xnorm_hist[ka], 1e-300);
        convert_mat(S->b[best_pair[1]], Xa64, s);
        eb = std::sqrt(e2_sq(c, A64, Xa64, s)) / std::max(xnorm_hist[kb], 1e-300);
      }
      if (best_j - 1 >= 1 && ea < eb) {
        chosen_buf = best_pair[0];
        chosen_j = best_j - 1;
      } else {
        chosen_buf = best_pair[1];
        chosen_j = best_j;
      }
    } else if (dec == D_NEWMIN) {
      best_pair[0] = cur;
      best_pair[1] = nxt;
      best_j = j;
    }
    if (reason >= 0) {
      inf.stop_reason = reason;
      if (has_finish) {
        // continue in FP64 from the chosen iterate
        ++ph;
        const int dt2 = store_of(phases[ph]);
        IterSet* S2 = &set_of(dt2);
        if (dt2 != dt) {
          convert_mat(S->b[chosen_buf], S2->b[0], s);
          cur = 0;
        } else {
          cur = chosen_buf;
        }
        S = S2;
        dt = dt2;
        best_pair[0] = best_pair[1] = -1;
        j = chosen_j;
        xnorm_hist.resize(j + 1);
        returned_buf = cur;
        returned_j = j;
        continue;
      }
      returned_buf = chosen_buf;
      returned_j = chosen_j;
      done = true;
      continue;
    }
    cur = nxt;
  }

  inf.iters = inf.iters_bf16 + inf.iters_f32 + inf.iters_f64;
  inf.returned = returned_j;
  Mat Xret = S->b[returned_buf];
  if (c.opt.penrose_finish && status != QPINV_EDIVERGED && !(c.opt.penrose_finish == 2 && has_finish)) {
    // X A X after the last update (any precision), or for FP64 solves the projection followed by one FP64
    // Newton-Schulz update (the same order as inside the finish)
    Mat X64 = Xret;
    if (X64.dtype != QPINV_F64) {
      Mat t = ws_mat(c, "pf_x", n, m, QPINV_F64);
      convert_mat(X64, t, s);
      X64 = t;
    }
    Mat O = ws_mat(c, "pf_out", n, m, QPINV_F64);
    const Mat A64 = A_of(QPINV_F64);
    penrose_project(c, c.opt.penrose_finish, A64, X64, O, s);
    if (c.opt.penrose_finish == 2) {
      Mat N = ws_mat(c, "pf_ns", n, m, QPINV_F64);
      chain(c, QPINV_NS, 2, side, P_F64, A64, O, N, nullptr, s);
      ++inf.iters_f64;
      ++inf.iters;
      ++inf.returned;
      O = N;
    }
    Xret = O;
  }
  convert_mat(Xret, Xout, s);
  QP_HIP(hipStreamSynchronize(s));
  return finish(status);
}

// ------------------------------------------------------------------------------------------------
// batched solves: one persistent launch per batch (batched.hip)
// ------------------------------------------------------------------------------------------------
int solve_batched(Ctx& c, int method, int order, int batch, const qpinv_qmat* A, qpinv_qmat* X, int scaling,
                  const double* alpha, double tol, int max_iter, int stop, qpinv_info* infos, hipStream_t s) {
  const double t0 = now_s();
  check_method(method, order);
  if (method != QPINV_NS && method != QPINV_QSAI && method != QPINV_QHPI19)
    throw Error(QPINV_EINVAL, "batched solves support NS, QSAI and QHPI19");
  if (batch < 0 || (batch > 0 && (!A || !X))) throw Error(QPINV_EINVAL, "bad batch arrays");
  if (scaling != QPINV_ALPHA_POWER && scaling != QPINV_ALPHA_GIVEN)
    throw Error(QPINV_EINVAL, "batched solves take ALPHA_POWER or ALPHA_GIVEN");
  if (scaling == QPINV_ALPHA_GIVEN && !alpha) throw Error(QPINV_EINVAL, "ALPHA_GIVEN needs the alpha array");
  if (!(tol >= 0.0) || max_iter < 1) throw Error(QPINV_EINVAL, "tol must be >= 0 and max_iter >= 1");
  if (stop != STOP_DX_ABS && stop != STOP_DX_REL && stop != STOP_GUARDED)
    throw Error(QPINV_EINVAL, "batched solves take the DX_ABS, DX_REL or GUARDED stop rule");
  if (batch == 0) return QPINV_OK;
  std::vector<BDesc> desc(batch);
  std::vector<double> work(batch);
  int64_t D = 8;
  for (int b = 0; b < batch; ++b) {
    validate(&A[b], "A[b]");
    validate(&X[b], "X[b]");
    if (A[b].dtype != QPINV_F32 || X[b].dtype != QPINV_F32) throw Error(QPINV_EINVAL, "batched solves use FP32 storage");
    const int64_t m = A[b].rows, n = A[b].cols;
    if (m < 1 || n < 1 || m > 512 || n > 512) throw Error(QPINV_EINVAL, "batched matrices must have 1..512 rows and cols");
    if (X[b].rows != n || X[b].cols != m) throw Error(QPINV_EINVAL, "X[b] must be n x m");
    if (scaling == QPINV_ALPHA_GIVEN && !(alpha[b] > 0.0)) throw Error(QPINV_EINVAL, "alpha[b] must be > 0");
    desc[b] = BDesc{static_cast<const float*>(A[b].data), A[b].ld, A[b].plane_stride, static_cast<float*>(X[b].data),
                    X[b].ld, X[b].plane_stride, (int)m, (int)n};
    const double sd = (double)std::min(m, n), od = (double)std::max(m, n);
    work[b] = sd * sd * od;
    D = std::max<int64_t>(D, std::max(m, n));
  }
  D = round8(D);
  // largest work first
  std::vector<int> order_v(batch);
  for (int b = 0; b < batch; ++b) order_v[b] = b;
  std::stable_sort(order_v.begin(), order_v.end(), [&](int a, int b2) { return work[a] > work[b2]; });
  std::vector<double> alphas;
  if (scaling == QPINV_ALPHA_GIVEN) alphas.assign(alpha, alpha + batch);
  BKey key;
  key.count = batch;
  key.D = (int)D;
  key.method = method == QPINV_NS ? 0 : method == QPINV_QSAI ? 2 : 3;
  key.stop = stop;
  key.max_iter = max_iter;
  key.tol = tol;
  key.scaling = scaling == QPINV_ALPHA_GIVEN ? 2 : 0;
  key.power_steps = c.opt.power_steps;
  key.seed = c.opt.power_seed;
  key.dyn = c.opt.batched_dynamic;
  if (!c.batched) c.batched = new BatchedState();
  std::vector<BInfo> out;
  // tile configuration: tuned per batch signature (size histogram) when autotuning is on
  std::vector<int64_t> sig = {batch, D, key.method, stop, max_iter};
  for (int b = 0; b < batch; ++b) {
    sig.push_back(A[b].rows);
    sig.push_back(A[b].cols);
  }
  auto usable = [&](int cfg) { return !batched_is_sync(cfg) || batch <= 2048; };
  auto it = c.batched_tuned.find(sig);
  if (c.opt.batched_cfg >= 0) {
    if (!usable(c.opt.batched_cfg)) throw Error(QPINV_EINVAL, "batched configuration takes at most 2048 matrices");
    key.cfg = c.opt.batched_cfg;
  } else if (it != c.batched_tuned.end()) {
    key.cfg = it->second;
  } else if (c.opt.autotune) {
    double best = 1e300;
    int best_cfg = 0;
    for (int cfg = 0; cfg < batched_num_configs(); ++cfg) {
      if (!usable(cfg)) continue;
      key.cfg = cfg;
      run_batched(*c.batched, key, desc, order_v, alphas, out, s);  // builds the graph (and warms up)
      const double t1 = now_s();
      run_batched(*c.batched, key, desc, order_v, alphas, out, s);
      const double dt = now_s() - t1;
      if (c.opt.verbose) fprintf(stderr, "[qpinv] batched %s: %.3f ms\n", batched_config_name(cfg), 1e3 * dt);
      if (dt < best) {
        best = dt;
        best_cfg = cfg;
      }
    }
    key.cfg = best_cfg;
    c.batched_tuned[sig] = best_cfg;
  } else {
    // measured on the 512-matrix workload: phase-synchronous 32 x 32 x 32 tiles first, then the
    // queue form with 64 x 64 tiles (batches above the phase-synchronous limit)
    key.cfg = usable(kBatchedDefaultSync) ? kBatchedDefaultSync : kBatchedDefaultQueue;
  }
  run_batched(*c.batched, key, desc, order_v, alphas, out, s, c.opt.verbose != 0);
  const double secs = now_s() - t0;
  int status = QPINV_OK;
  for (int b = 0; b < batch; ++b) {
    const BInfo& bi = out[b];
    if (infos) {
      qpinv_info& r = infos[b];
      std::memset(&r, 0, sizeof(r));
      r.iters = bi.iters;
      r.iters_f32 = bi.iters;
      r.returned = bi.returned;
      r.stop_reason = bi.reason;
      r.side = desc[b].m > desc[b].n ? QPINV_SIDE_LEFT : QPINV_SIDE_RIGHT;
      r.alpha_used = bi.alpha;
      r.mu_used = bi.sigma1_sq > 0 ? bi.alpha * bi.sigma1_sq : 0.0;
      r.sigma1_sq_est = bi.sigma1_sq;
      r.final_dx_rel = bi.dx_rel;
      r.e1_rel = -1.0;
      r.seconds = secs;
      r.reserved = bi.status;
    }
    if (bi.status == QPINV_ENONFINITE || bi.status == QPINV_EDIVERGED)
      status = status == QPINV_OK || status == QPINV_ENOTCONVERGED ? bi.status : status;
    else if (bi.status == QPINV_ENOTCONVERGED && status == QPINV_OK)
      status = QPINV_ENOTCONVERGED;
  }
  return status;
}

// ------------------------------------------------------------------------------------------------
// Penrose residuals in FP64 (Section 4 error metrics)
// ------------------------------------------------------------------------------------------------
void residuals(Ctx& c, const qpinv_qmat* Aq, const qpinv_qmat* Xq, double E_abs[4], double E_rel[4], hipStream_t s) {
  validate(Aq, "A");
  validate(Xq, "X");
  if (Xq->rows != Aq->cols || Xq->cols != Aq->rows) throw Error(QPINV_EINVAL, "X must be n x m for A m x n");
  const Mat A0 = from_abi(*Aq), X0 = from_abi(*Xq);
  const int64_t m = A0.rows, n = A0.cols;
  for (int k = 0; k < 4; ++k) E_abs[k] = E_rel[k] = 0.0;
  if (m == 0 || n == 0) return;
  Mat A = A0, X = X0;
  if (A0.dtype != QPINV_F64) {
    A = ws_mat(c, "resA", m, n, QPINV_F64);
    convert_mat(A0, A, s);
  }
  if (X0.dtype != QPINV_F64) {
    X = ws_mat(c, "resX", n, m, QPINV_F64);
    convert_mat(X0, X, s);
  }
  Mat AX = ws_mat(c, "res_ax", m, m, QPINV_F64);
  Mat XA = ws_mat(c, "res_xa", n, n, QPINV_F64);
  Mat O1 = ws_mat(c, "res_o1", m, n, QPINV_F64);
  Mat O2 = ws_mat(c, "res_o2", n, m, QPINV_F64);
  double* d = c.dsc + 32;
  gemm(c, P_F64, A, X, epi1(AX), s);
  gemm(c, P_F64, X, A, epi1(XA), s);
  {
    Epilogue e = epi1(O1);
    e.nin = 1;
    e.in[0] = A.v;
    e.b[0][0] = -1.0;
    e.reduce = true;
    gemm(c, P_F64, AX, A, e, s, d);  // d[0] = ||AXA - A||^2
  }
  {
    Epilogue e = epi1(O2);
    e.nin = 1;
    e.in[0] = X.v;
    e.b[0][0] = -1.0;
    e.reduce = true;
    gemm(c, P_F64, XA, X, e, s, d + 2);  // d[2] = ||XAX - X||^2
  }
  double* work = static_cast<double*>(c.ws.get("hermwork", sizeof(double) * 2 * hermdiff_blocks(std::max(m, n))));
  herm_diff<double>(AX.v, m, d + 4, work, s);
  herm_diff<double>(XA.v, n, d + 6, work, s);
  double* nw = static_cast<double*>(
      c.ws.get("normwork", sizeof(double) * std::max(norms_work_doubles(m, n), norms_work_doubles(n, m))));
  norms<double>(A.v, m, n, d + 8, nw, s);
  norms<double>(X.v, n, m, d + 12, nw, s);
  to_host(c, d, 16, s);
  const double* h = c.hsc;
  E_abs[0] = std::sqrt(h[0]);
  E_abs[1] = std::sqrt(h[2]);
  E_abs[2] = std::sqrt(h[4]);
  E_abs[3] = std::sqrt(h[6]);
  const double nA = std::sqrt(h[8]), nX = std::sqrt(h[12]), nAX = std::sqrt(h[5]), nXA = std::sqrt(h[7]);
  E_rel[0] = nA > 0 ? E_abs[0] / nA : 0.0;
  E_rel[1] = nX > 0 ? E_abs[1] / nX : 0.0;
  E_rel[2] = nAX > 0 ? E_abs[2] / nAX : 0.0;
  E_rel[3] = nXA > 0 ? E_abs[3] / nXA : 0.0;
}

void features(Ctx& c, const Mat& A, int steps, double out[7], hipStream_t s) {
  double nh[4];
  norms_host(c, A, nh, s);
  if (nh[3] > 0) throw Error(QPINV_ENONFINITE, "A holds NaN or Inf");
  out[0] = power_host(c, A, steps > 0 ? steps : c.opt.power_steps, s, &out[6]);
  out[1] = std::sqrt(nh[0]);
  out[2] = nh[1];
  out[3] = nh[2];
  out[4] = (double)A.rows;
  out[5] = (double)A.cols;
}

// ------------------------------------------------------------------------------------------------
// autotuner: time every tile configuration on the shape, keep the fastest
// ------------------------------------------------------------------------------------------------
int autotune(Ctx& c, Prec p, int64_t M, int64_t N, int64_t K, double* best_ms, hipStream_t s) {
  if (M < 1 || N < 1 || K < 1) throw Error(QPINV_EINVAL, "autotune: empty shape");
  const int dt = store_of(p);
  Mat A = ws_mat(c, "tuneA", M, K, dt), B = ws_mat(c, "tuneB", K, N, dt), C = ws_mat(c, "tuneC", M, N, dt);
  const size_t es = esize(dt);
  if (es == 8) {
    fill_pattern(static_cast<double*>(A.v.p), 4 * A.v.ps, s);
    fill_pattern(static_cast<double*>(B.v.p), 4 * B.v.ps, s);
  } else {
    fill_pattern(static_cast<float*>(A.v.p), 4 * A.v.ps, s);
    fill_pattern(static_cast<float*>(B.v.p), 4 * B.v.ps, s);
  }
  const int ncfg = (int)tile_configs(p).size();
  hipEvent_t e0, e1;
  QP_HIP(hipEventCreate(&e0));
  QP_HIP(hipEventCreate(&e1));
  int best = default_config(p, M, N, K);
  double best_t = 1e300;
  // two timed rounds over all configurations (the first also warms clocks and caches); a
  // configuration's time is its faster round
  const int reps = 3;
  std::vector<double> tbest(ncfg, 1e300);
  for (int round = 0; round < 2; ++round)
    for (int cfg = 0; cfg < ncfg; ++cfg) {
      qgemm(p, A.v, B.v, M, N, K, epi1(C), nullptr, c.scratch, s, cfg);  // warm-up
      QP_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) qgemm(p, A.v, B.v, M, N, K, epi1(C), nullptr, c.scratch, s, cfg);
      QP_HIP(hipEventRecord(e1, s));
      QP_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      QP_HIP(hipEventElapsedTime(&ms, e0, e1));
      tbest[cfg] = std::min(tbest[cfg], (double)ms / reps);
    }
  for (int cfg = 0; cfg < ncfg; ++cfg) {
    const double t = tbest[cfg];
    if (c.opt.verbose) fprintf(stderr, "[qpinv] tune %s %ldx%ldx%ld: %.4f ms\n", tile_configs(p)[cfg].name, (long)M, (long)N, (long)K, t);
    if (t < best_t) {
      best_t = t;
      best = cfg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c.tuned[std::make_tuple((int)p, M, N, K)] = best;
  if (best_ms) *best_ms = best_t;
  return best;
}

}  // namespace qp

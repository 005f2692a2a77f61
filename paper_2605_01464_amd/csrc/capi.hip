// extern "C" boundary of libqpinv.so: argument checks, error codes, no exceptions across the ABI.
#include <cstring>
#include <fstream>
#include <iterator>
#include <string>

#include "../../include/qpinv.h"
#include "apps.hpp"
#include "aux.hpp"
#include "batched.hpp"
#include "controller.hpp"
#include "krylov.hpp"
#include "mlp.hpp"
#include "solver.hpp"
#include "tunecache.hpp"

struct qpinv_ctx {
  qp::Ctx* impl;
};

namespace {
thread_local std::string g_last_error;

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const qp::Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return QPINV_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return QPINV_EHIP;
  } catch (...) {
    g_last_error = "unknown error";
    return QPINV_EHIP;
  }
}

qp::Ctx& ctx_of(qpinv_ctx* c) {
  if (!c || !c->impl) throw qp::Error(QPINV_EINVAL, "null context");
  QP_HIP(hipSetDevice(c->impl->device));
  return *c->impl;
}

hipStream_t stream_of(void* s) { return static_cast<hipStream_t>(s); }

int prec_check(int gemm_prec) {
  if (gemm_prec < QPINV_GEMM_F64 || gemm_prec > QPINV_GEMM_BF16X3) throw qp::Error(QPINV_EINVAL, "bad product precision");
  return gemm_prec;
}

int storage_for(int gemm_prec) { return gemm_prec == QPINV_GEMM_F64 ? QPINV_F64 : QPINV_F32; }

// The device token of a tune cache: architecture name and compute-unit count.
std::string tune_device(int dev) {
  hipDeviceProp_t pr{};
  QP_HIP(hipGetDeviceProperties(&pr, dev));
  return std::string(pr.gcnArchName) + ":" + std::to_string(pr.multiProcessorCount) + "cu";
}

void set_option(qp::Ctx& c, const std::string& key, double v) {
  auto need = [&](bool ok) {
    if (!ok) throw qp::Error(QPINV_EINVAL, "option " + key + ": value out of range");
  };
  if (key == "side") {
    need(v == 0 || v == 1 || v == 2);
    c.opt.side = (int)v;
  } else if (key == "power_steps") {
    need(v >= 1 && v <= 1000);
    c.opt.power_steps = (int)v;
  } else if (key == "power_seed") {
    need(v >= 0);
    c.opt.power_seed = (uint64_t)v;
  } else if (key == "autotune") {
    need(v == 0 || v == 1);
    c.opt.autotune = (int)v;
  } else if (key == "f64_refined") {
    need(v == 0 || v == 1);
    c.opt.f64_refined = (int)v;
  } else if (key == "finish_method") {
    need(v == -1 || v == QPINV_NS || v == QPINV_QSAI || v == QPINV_QHPI19);
    c.opt.finish_method = (int)v;
  } else if (key == "small_path") {
    need(v == 0 || v == 1);
    c.opt.small_path = (int)v;
  } else if (key == "small_gram") {
    need(v == 0 || v == 1);
    c.opt.small_gram = (int)v;
  } else if (key == "fault_small_giveup") {
    need(v == 0 || v == 1);
    c.opt.fault_small_giveup = (int)v;
  } else if (key == "penrose_finish") {
    need(v == 0 || v == 1 || v == 2);
    c.opt.penrose_finish = (int)v;
  } else if (key == "f64_finish_iters") {
    need(v >= 1 && v <= 4);
    c.opt.f64_finish_iters = (int)v;
  } else if (key == "mixed_switch") {
    need(v > 0 && v < 1);
    c.opt.mixed_switch = v;
  } else if (key == "mixed_rnorm_steps") {
    need(v >= 1 && v <= 100);
    c.opt.mixed_rnorm_steps = (int)v;
  } else if (key == "max_bf16_iters") {
    need(v >= 0 && v <= 100);
    c.opt.max_bf16_iters = (int)v;
  } else if (key == "mixed_split") {
    need(v == 0 || v == 1);
    c.opt.mixed_split = (int)v;
  } else if (key == "gemm_timing") {
    need(v == 0 || v == 1);
    c.opt.gemm_timing = (int)v;
  } else if (key == "gemm_cfg_f64" || key == "gemm_cfg_f32" || key == "gemm_cfg_bf16" || key == "gemm_cfg_bf16x3") {
    const qp::Prec p = key == "gemm_cfg_f64"    ? qp::P_F64
                       : key == "gemm_cfg_f32"  ? qp::P_F32
                       : key == "gemm_cfg_bf16" ? qp::P_BF16
                                                : qp::P_BF16X3;
    need(v == -1 || (v >= 0 && v < (double)qp::tile_configs(p).size() && v == (int)v));
    c.opt.force_cfg[(int)p] = (int)v;
  } else if (key == "batched_cfg") {
    need(v == -1 || (v >= 0 && v < (double)qp::batched_num_configs() && v == (int)v));
    c.opt.batched_cfg = (int)v;
  } else if (key == "batched_dynamic") {
    need(v == 0 || v == 1);
    c.opt.batched_dynamic = (int)v;
  } else if (key == "verbose") {
    c.opt.verbose = v != 0;
  } else {
    throw qp::Error(QPINV_EINVAL, "unknown option " + key);
  }
}
}  // namespace

extern "C" {

const char* qpinv_strerror(int status) {
  switch (status) {
    case QPINV_OK: return "ok";
    case QPINV_EINVAL: return "invalid argument";
    case QPINV_ENONFINITE: return "non-finite input";
    case QPINV_EDIVERGED: return "iteration diverged";
    case QPINV_ENOTCONVERGED: return "not converged within max_iter";
    case QPINV_EHIP: return "HIP runtime error";
    case QPINV_ENOMEM: return "out of memory";
    case QPINV_ETIMEOUT: return "bounded wait expired";
    default: return "unknown status";
  }
}

const char* qpinv_last_error(void) { return g_last_error.c_str(); }

int qpinv_init(qpinv_ctx** out, int device, const char* config) {
  return guarded([&]() {
    if (!out) throw qp::Error(QPINV_EINVAL, "null output pointer");
    *out = nullptr;
    int count = 0;
    QP_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) throw qp::Error(QPINV_EINVAL, "no such device");
    auto* impl = new qp::Ctx(device);
    try {
      if (config) {
        std::string cfg(config);
        size_t pos = 0;
        while (pos < cfg.size()) {
          size_t end = cfg.find(';', pos);
          if (end == std::string::npos) end = cfg.size();
          std::string item = cfg.substr(pos, end - pos);
          pos = end + 1;
          if (item.empty()) continue;
          const size_t eq = item.find('=');
          if (eq == std::string::npos) throw qp::Error(QPINV_EINVAL, "config item without '=': " + item);
          char* tail = nullptr;
          const std::string val = item.substr(eq + 1);
          const double v = std::strtod(val.c_str(), &tail);
          if (!tail || *tail != '\0') throw qp::Error(QPINV_EINVAL, "config value not numeric: " + item);
          set_option(*impl, item.substr(0, eq), v);
        }
      }
    } catch (...) {
      delete impl;
      throw;
    }
    *out = new qpinv_ctx{impl};
    return QPINV_OK;
  });
}

int qpinv_set_option(qpinv_ctx* c, const char* key, double value) {
  return guarded([&]() {
    if (!key) throw qp::Error(QPINV_EINVAL, "null key");
    set_option(ctx_of(c), key, value);
    return QPINV_OK;
  });
}

int qpinv_finalize(qpinv_ctx* c) {
  return guarded([&]() {
    if (!c) return QPINV_OK;
    if (c->impl) qp::mlp_free(c->impl);
    delete c->impl;
    delete c;
    return QPINV_OK;
  });
}

int qpinv_solve(qpinv_ctx* c, int method, int order, const qpinv_qmat* A, int scaling, double alpha_or_mu, double tol,
                int max_iter, int stop, int precision, qpinv_qmat* X, qpinv_info* info, void* hip_stream) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    return qp::solve(cx, method, order, A, scaling, alpha_or_mu, tol, max_iter, stop, precision, X, info,
                     stream_of(hip_stream));
  });
}

int qpinv_solve_noalloc(qpinv_ctx* c, int method, int order, const qpinv_qmat* A, int scaling, double alpha_or_mu,
                        double tol, int max_iter, int stop, int precision, qpinv_qmat* X, qpinv_info* info,
                        void* hip_stream) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    return qp::solve_noalloc(cx, method, order, A, scaling, alpha_or_mu, tol, max_iter, stop, precision, X, info,
                             stream_of(hip_stream));
  });
}

int qpinv_solve_batched(qpinv_ctx* c, int method, int order, int batch, const qpinv_qmat* A, qpinv_qmat* X,
                        int scaling, const double* alpha, double tol, int max_iter, int stop, qpinv_info* infos,
                        void* hip_stream) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    return qp::solve_batched(cx, method, order, batch, A, X, scaling, alpha, tol, max_iter, stop, infos,
                             stream_of(hip_stream));
  });
}

int qpinv_step(qpinv_ctx* c, int method, int order, int side, int gemm_prec, const qpinv_qmat* A, const qpinv_qmat* X_in,
               qpinv_qmat* X_out, double dx[2], void* hip_stream) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    prec_check(gemm_prec);
    qp::check_method(method, order);
    qp::validate(A, "A");
    qp::validate(X_in, "X_in");
    qp::validate(X_out, "X_out");
    const int st = storage_for(gemm_prec);
    if (A->dtype != st || X_in->dtype != st || X_out->dtype != st)
      throw qp::Error(QPINV_EINVAL, "step: A and X must have the storage type of the product precision");
    if (X_in->rows != A->cols || X_in->cols != A->rows || X_out->rows != A->cols || X_out->cols != A->rows)
      throw qp::Error(QPINV_EINVAL, "step: X must be n x m");
    if (X_in->data == X_out->data && X_in->rows * X_in->cols > 0) throw qp::Error(QPINV_EINVAL, "step: X_out aliases X_in");
    if (side != QPINV_SIDE_LEFT && side != QPINV_SIDE_RIGHT && side != QPINV_SIDE_AUTO)
      throw qp::Error(QPINV_EINVAL, "bad side");
    if (side == QPINV_SIDE_AUTO) side = A->rows > A->cols ? QPINV_SIDE_LEFT : QPINV_SIDE_RIGHT;
    if (A->rows == 0 || A->cols == 0) {
      if (dx) dx[0] = dx[1] = 0.0;
      return QPINV_OK;
    }
    hipStream_t s = stream_of(hip_stream);
    qp::chain(cx, method, order, side, (qp::Prec)gemm_prec, qp::from_abi(*A), qp::from_abi(*X_in),
              qp::from_abi(*X_out), cx.dsc, s);
    QP_HIP(hipMemcpyAsync(cx.hsc, cx.dsc, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    QP_HIP(hipStreamSynchronize(s));
    if (dx) {
      dx[0] = cx.hsc[0];
      dx[1] = cx.hsc[1];
    }
    return QPINV_OK;
  });
}

int qpinv_residuals(qpinv_ctx* c, const qpinv_qmat* A, const qpinv_qmat* X, double E_abs[4], double E_rel[4],
                    void* hip_stream) {
  return guarded([&]() {
    if (!E_abs || !E_rel) throw qp::Error(QPINV_EINVAL, "null output arrays");
    qp::residuals(ctx_of(c), A, X, E_abs, E_rel, stream_of(hip_stream));
    return QPINV_OK;
  });
}

static int qgemm_impl(qpinv_ctx* c, int gemm_prec, int cfg, const qpinv_qmat* A, const qpinv_qmat* B, qpinv_qmat* C,
                      double alpha, double beta, double gamma, void* hip_stream) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    prec_check(gemm_prec);
    qp::validate(A, "A");
    qp::validate(B, "B");
    qp::validate(C, "C");
    const int st = storage_for(gemm_prec);
    if (A->dtype != st || B->dtype != st || C->dtype != st)
      throw qp::Error(QPINV_EINVAL, "qgemm: operands must have the storage type of the product precision");
    if (A->cols != B->rows || C->rows != A->rows || C->cols != B->cols) throw qp::Error(QPINV_EINVAL, "qgemm: shape mismatch");
    if (C->data && (C->data == A->data || C->data == B->data)) throw qp::Error(QPINV_EINVAL, "qgemm: C aliases an operand");
    const int ncfg = (int)qp::tile_configs((qp::Prec)gemm_prec).size();
    if (cfg >= ncfg) throw qp::Error(QPINV_EINVAL, "qgemm: bad tile configuration");
    const qp::Mat Am = qp::from_abi(*A), Bm = qp::from_abi(*B), Cm = qp::from_abi(*C);
    qp::Epilogue e;
    e.nout = 1;
    e.out[0] = Cm.v;
    e.a[0] = alpha;
    e.g[0] = gamma;
    if (beta != 0.0) {
      e.nin = 1;
      e.in[0] = Cm.v;
      e.b[0][0] = beta;
    }
    const int64_t M = A->rows, N = B->cols, K = A->cols;
    if (cfg < 0) cfg = cx.config_for((qp::Prec)gemm_prec, M, N, K, stream_of(hip_stream));
    cx.flops += 32.0 * (double)M * (double)N * (double)K;
    qp::qgemm((qp::Prec)gemm_prec, Am.v, Bm.v, M, N, K, e, nullptr, cx.scratch, stream_of(hip_stream), cfg);
    return QPINV_OK;
  });
}

int qpinv_qgemm(qpinv_ctx* c, int gemm_prec, const qpinv_qmat* A, const qpinv_qmat* B, qpinv_qmat* C, double alpha,
                double beta, double gamma, void* hip_stream) {
  return qgemm_impl(c, gemm_prec, -1, A, B, C, alpha, beta, gamma, hip_stream);
}

int qpinv_qgemm_cfg(qpinv_ctx* c, int gemm_prec, int cfg, const qpinv_qmat* A, const qpinv_qmat* B, qpinv_qmat* C,
                    double alpha, double beta, double gamma, void* hip_stream) {
  if (cfg < 0) {
    g_last_error = "qgemm_cfg: cfg must be >= 0";
    return QPINV_EINVAL;
  }
  return qgemm_impl(c, gemm_prec, cfg, A, B, C, alpha, beta, gamma, hip_stream);
}

int qpinv_x0(qpinv_ctx* c, const qpinv_qmat* A, double alpha, qpinv_qmat* X, void* hip_stream) {
  return guarded([&]() {
    ctx_of(c);
    qp::validate(A, "A");
    qp::validate(X, "X");
    if (X->rows != A->cols || X->cols != A->rows) throw qp::Error(QPINV_EINVAL, "x0: X must be n x m");
    const qp::Mat Am = qp::from_abi(*A), Xm = qp::from_abi(*X);
    hipStream_t s = stream_of(hip_stream);
    if (Am.dtype == QPINV_F32 && Xm.dtype == QPINV_F32)
      qp::x0_scaled_adjoint<float, float>(Am.v, Am.rows, Am.cols, alpha, Xm.v, s);
    else if (Am.dtype == QPINV_F32)
      qp::x0_scaled_adjoint<float, double>(Am.v, Am.rows, Am.cols, alpha, Xm.v, s);
    else if (Xm.dtype == QPINV_F32)
      qp::x0_scaled_adjoint<double, float>(Am.v, Am.rows, Am.cols, alpha, Xm.v, s);
    else
      qp::x0_scaled_adjoint<double, double>(Am.v, Am.rows, Am.cols, alpha, Xm.v, s);
    return QPINV_OK;
  });
}

int qpinv_submatrix(qpinv_ctx* c, const qpinv_qmat* A, const int* rows, int nrows, const int* cols, int ncols,
                    qpinv_qmat* B, void* hip_stream) {
  return guarded([&]() {
    ctx_of(c);
    qp::validate(A, "A");
    qp::validate(B, "B");
    if (nrows < 0 || ncols < 0) throw qp::Error(QPINV_EINVAL, "submatrix: negative index count");
    if ((!rows && nrows != A->rows) || (!cols && ncols != A->cols))
      throw qp::Error(QPINV_EINVAL, "submatrix: a null index set selects all rows / columns");
    if (B->rows != nrows || B->cols != ncols) throw qp::Error(QPINV_EINVAL, "submatrix: B must be nrows x ncols");
    if (A->dtype != B->dtype) throw qp::Error(QPINV_EINVAL, "submatrix: A and B must share the dtype");
    const qp::Mat Am = qp::from_abi(*A), Bm = qp::from_abi(*B);
    hipStream_t s = stream_of(hip_stream);
    if (Am.dtype == QPINV_F32)
      qp::submatrix<float>(Am.v, Am.rows, Am.cols, rows, nrows, cols, ncols, Bm.v, s);
    else
      qp::submatrix<double>(Am.v, Am.rows, Am.cols, rows, nrows, cols, ncols, Bm.v, s);
    return QPINV_OK;
  });
}

int qpinv_masked_merge(qpinv_ctx* c, const qpinv_qmat* M, const unsigned char* mask, int64_t mask_ld,
                       const qpinv_qmat* X, qpinv_qmat* Y, void* hip_stream) {
  return guarded([&]() {
    ctx_of(c);
    qp::validate(M, "M");
    qp::validate(X, "X");
    qp::validate(Y, "Y");
    if (M->rows != X->rows || M->cols != X->cols || Y->rows != X->rows || Y->cols != X->cols)
      throw qp::Error(QPINV_EINVAL, "masked_merge: M, X and Y must have one shape");
    if (M->dtype != X->dtype || Y->dtype != X->dtype) throw qp::Error(QPINV_EINVAL, "masked_merge: one dtype");
    if (!mask && X->rows > 0 && X->cols > 0) throw qp::Error(QPINV_EINVAL, "masked_merge: null mask");
    if (mask_ld < X->cols) throw qp::Error(QPINV_EINVAL, "masked_merge: mask_ld < cols");
    const qp::Mat Mm = qp::from_abi(*M), Xm = qp::from_abi(*X), Ym = qp::from_abi(*Y);
    hipStream_t s = stream_of(hip_stream);
    if (Xm.dtype == QPINV_F32)
      qp::masked_merge<float>(Mm.v, mask, mask_ld, Xm.v, Ym.v, Xm.rows, Xm.cols, s);
    else
      qp::masked_merge<double>(Mm.v, mask, mask_ld, Xm.v, Ym.v, Xm.rows, Xm.cols, s);
    return QPINV_OK;
  });
}

int qpinv_gl_krylov(qpinv_ctx* c, int method, const qpinv_qmat* A, const qpinv_qmat* B, const qpinv_qmat* M,
                    qpinv_qmat* X, double tol, int max_iter, int* iters, double* rr, double* true_rr, double* history,
                    int history_cap, void* hip_stream) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    if (method != QPINV_KRYLOV_FOM && method != QPINV_KRYLOV_GMRES) throw qp::Error(QPINV_EINVAL, "krylov: method");
    qp::validate(A, "A");
    qp::validate(B, "B");
    qp::validate(X, "X");
    if (M) qp::validate(M, "M");
    if (A->rows != A->cols || B->rows != A->rows || X->rows != A->cols || X->cols != B->cols ||
        (M && (M->rows != A->rows || M->cols != A->rows)))
      throw qp::Error(QPINV_EINVAL, "krylov: A n x n, B and X n x m, M n x n");
    if (A->dtype != QPINV_F64 || B->dtype != QPINV_F64 || X->dtype != QPINV_F64 || (M && M->dtype != QPINV_F64))
      throw qp::Error(QPINV_EINVAL, "krylov: FP64 matrices");
    if (X->cols > 1 && X->ld != X->cols) throw qp::Error(QPINV_EINVAL, "krylov: X must have ld = cols");
    if (X->plane_stride != X->rows * X->cols) throw qp::Error(QPINV_EINVAL, "krylov: X planes must be contiguous");
    if (max_iter < 1 || !(tol >= 0.0)) throw qp::Error(QPINV_EINVAL, "krylov: max_iter >= 1, tol >= 0");
    if (history_cap < 0 || (history_cap > 0 && !history)) throw qp::Error(QPINV_EINVAL, "krylov: history");
    if (A->rows == 0 || B->cols == 0) {
      if (iters) *iters = 0;
      if (rr) *rr = 0.0;
      if (true_rr) *true_rr = 0.0;
      return QPINV_OK;
    }
    const qp::Mat Am = qp::from_abi(*A), Bm = qp::from_abi(*B), Xm = qp::from_abi(*X);
    qp::Mat Mm;
    if (M) Mm = qp::from_abi(*M);
    const qp::KrylovResult r = qp::gl_krylov(cx, method, Am, Bm, M ? &Mm : nullptr, Xm, tol, max_iter, history,
                                             history_cap, stream_of(hip_stream));
    if (iters) *iters = r.iters;
    if (rr) *rr = r.rr;
    if (true_rr) *true_rr = r.true_rr;
    return r.status;
  });
}

int qpinv_features(qpinv_ctx* c, const qpinv_qmat* A, int power_steps, double out[7], void* hip_stream) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    if (!out) throw qp::Error(QPINV_EINVAL, "null output");
    qp::validate(A, "A");
    if (A->rows == 0 || A->cols == 0) throw qp::Error(QPINV_EINVAL, "features of an empty matrix");
    qp::features(cx, qp::from_abi(*A), power_steps, out, stream_of(hip_stream));
    return QPINV_OK;
  });
}

int qpinv_mlp_init(qpinv_ctx* c, uint64_t seed) {
  return guarded([&]() {
    qp::mlp_init(ctx_of(c), seed);
    return QPINV_OK;
  });
}

int qpinv_mlp_fit_normalization(qpinv_ctx* c, const double* raw, int count, void* hip_stream) {
  return guarded([&]() {
    if (!raw || count < 1) throw qp::Error(QPINV_EINVAL, "need raw features");
    qp::mlp_fit_normalization(ctx_of(c), raw, count, stream_of(hip_stream));
    return QPINV_OK;
  });
}

int qpinv_mlp_train_step(qpinv_ctx* c, const double* raw, const double* target, const int* idx, int batch, double lr,
                         double* loss, void* hip_stream) {
  return guarded([&]() {
    if (!raw || !target || batch < 1 || batch > 1024 || !(lr > 0.0)) throw qp::Error(QPINV_EINVAL, "bad training step");
    const double l = qp::mlp_train_step(ctx_of(c), raw, target, idx, batch, lr, nullptr, stream_of(hip_stream));
    if (loss) *loss = l;
    return QPINV_OK;
  });
}

int qpinv_mlp_gradient(qpinv_ctx* c, const double* raw, const double* target, int batch, float* grad, double* loss,
                       void* hip_stream) {
  return guarded([&]() {
    if (!raw || !target || !grad || batch < 1 || batch > 1024) throw qp::Error(QPINV_EINVAL, "bad gradient request");
    const double l = qp::mlp_train_step(ctx_of(c), raw, target, nullptr, batch, 1.0, grad, stream_of(hip_stream));
    if (loss) *loss = l;
    return QPINV_OK;
  });
}

int qpinv_mlp_predict(qpinv_ctx* c, const double* raw, int count, double* mu, void* hip_stream) {
  return guarded([&]() {
    if (!raw || !mu || count < 0) throw qp::Error(QPINV_EINVAL, "bad prediction request");
    qp::mlp_predict(ctx_of(c), raw, count, mu, stream_of(hip_stream));
    return QPINV_OK;
  });
}

int qpinv_mlp_num_params(void) { return qp::mlp_num_params(); }

int qpinv_mlp_get_params(qpinv_ctx* c, float* host, int n) {
  int need = 0;
  const int st = guarded([&]() {
    need = qp::mlp_get(ctx_of(c), host, n);
    return QPINV_OK;
  });
  return st == QPINV_OK ? need : st;
}

int qpinv_mlp_set_params(qpinv_ctx* c, const float* host, int n) {
  return guarded([&]() {
    qp::mlp_set(ctx_of(c), host, n);
    return QPINV_OK;
  });
}

int qpinv_spectral_labels(qpinv_ctx* c, int method, int order, const double* spectra, const int* offsets, int count,
                          const double* s1sq_est, double tol, int max_iter, int ngrid, double mu_lo, double mu_hi,
                          double mu_target, double* mu_out, int* j_best, int* j_classical, void* hip_stream) {
  return guarded([&]() {
    qp::check_method(method, order);
    if (count < 0 || (count > 0 && (!spectra || !offsets || !s1sq_est || !mu_out || !j_best || !j_classical)) ||
        !(tol > 0.0) || max_iter < 1 || max_iter > 64)
      throw qp::Error(QPINV_EINVAL, "bad label request");
    qp::spectral_labels(ctx_of(c), method, order, spectra, offsets, count, s1sq_est, tol, max_iter, ngrid, mu_lo, mu_hi,
                        mu_target, mu_out, j_best, j_classical, stream_of(hip_stream));
    return QPINV_OK;
  });
}

int qpinv_autotune(qpinv_ctx* c, int gemm_prec, int64_t M, int64_t N, int64_t K, double* best_ms, void* hip_stream) {
  int cfg = -1;
  const int st = guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    prec_check(gemm_prec);
    cfg = qp::autotune(cx, (qp::Prec)gemm_prec, M, N, K, best_ms, stream_of(hip_stream));
    return QPINV_OK;
  });
  return st == QPINV_OK ? cfg : st;
}

int qpinv_tune_save(qpinv_ctx* c, const char* path) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    if (!path || !*path) throw qp::Error(QPINV_EINVAL, "tune cache: no path");
    qp::TuneFile f;
    f.device = tune_device(cx.device);
    for (const auto& e : cx.tuned) {
      const int p = std::get<0>(e.first);
      f.gemm.emplace_back(p, std::get<1>(e.first), std::get<2>(e.first), std::get<3>(e.first),
                          qp::tile_configs((qp::Prec)p).at(e.second).name);
    }
    for (const auto& e : cx.batched_tuned) f.batched.emplace_back(e.first, qp::batched_config_name(e.second));
    std::ofstream out(path, std::ios::binary | std::ios::trunc);
    out << qp::tune_format(f);
    out.close();
    if (!out) throw qp::Error(QPINV_EINVAL, std::string("tune cache: cannot write ") + path);
    return (int)(f.gemm.size() + f.batched.size());
  });
}

int qpinv_tune_load(qpinv_ctx* c, const char* path) {
  return guarded([&]() {
    qp::Ctx& cx = ctx_of(c);
    if (!path || !*path) throw qp::Error(QPINV_EINVAL, "tune cache: no path");
    std::ifstream in(path, std::ios::binary);
    if (!in) throw qp::Error(QPINV_EINVAL, std::string("tune cache: cannot read ") + path);
    const std::string text((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    qp::TuneFile f;
    std::string err;
    if (!qp::tune_parse(text, f, err)) throw qp::Error(QPINV_EINVAL, err);
    if (f.device != tune_device(cx.device)) return 0;
    // names to indices; entries whose configuration this library does not have are skipped
    int applied = 0;
    for (const auto& g : f.gemm) {
      const auto& t = qp::tile_configs((qp::Prec)std::get<0>(g));
      for (int k = 0; k < (int)t.size(); ++k)
        if (std::get<4>(g) == t[k].name) {
          cx.tuned[std::make_tuple(std::get<0>(g), std::get<1>(g), std::get<2>(g), std::get<3>(g))] = k;
          ++applied;
          break;
        }
    }
    for (const auto& b : f.batched)
      for (int k = 0; k < qp::batched_num_configs(); ++k)
        if (b.second == qp::batched_config_name(k)) {
          cx.batched_tuned[b.first] = k;
          ++applied;
          break;
        }
    return applied;
  });
}

int qpinv_num_tile_configs(int gemm_prec) {
  if (gemm_prec < QPINV_GEMM_F64 || gemm_prec > QPINV_GEMM_BF16X3) return QPINV_EINVAL;
  return (int)qp::tile_configs((qp::Prec)gemm_prec).size();
}

const char* qpinv_tile_config_name(int gemm_prec, int cfg) {
  if (gemm_prec < QPINV_GEMM_F64 || gemm_prec > QPINV_GEMM_BF16X3) return "";
  const auto& t = qp::tile_configs((qp::Prec)gemm_prec);
  if (cfg < 0 || cfg >= (int)t.size()) return "";
  return t[cfg].name;
}

int qpinv_num_batched_configs(void) { return qp::batched_num_configs(); }

const char* qpinv_batched_config_name(int cfg) {
  if (cfg < 0 || cfg >= qp::batched_num_configs()) return "";
  return qp::batched_config_name(cfg);
}

int qpinv_gemm_stats(qpinv_ctx* c, double* out, int max_rows) {
  int rows = 0;
  const int st = guarded([&]() {
    if (!out || max_rows < 1) throw qp::Error(QPINV_EINVAL, "null output or max_rows < 1");
    rows = qp::gemm_stats(ctx_of(c), out, max_rows);
    return QPINV_OK;
  });
  return st == QPINV_OK ? rows : st;
}

int qpinv_controller_replay(int stop, double tol, int count, const double* d_abs, const double* x_norm,
                            const double* e1_rel, int* decision) {
  if (stop < qp::STOP_DX_ABS || stop > qp::STOP_GUARDED || count < 0 || !d_abs || !x_norm || !decision ||
      (stop == qp::STOP_E1_REL && !e1_rel) || !(tol >= 0.0)) {
    g_last_error = "controller_replay: bad argument";
    return QPINV_EINVAL;
  }
  qp::StopController ctl(stop, tol);
  for (int j = 0; j < count; ++j) {
    const int d = ctl.update(j + 1, d_abs[j], x_norm[j], e1_rel ? e1_rel[j] : -1.0);
    decision[j] = d;
    if (d == qp::D_TOL || d == qp::D_RISE || d == qp::D_DIVERGED) return j + 1;
  }
  return count;
}

}  // extern "C"

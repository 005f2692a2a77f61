// Allocation-free solve: qpinv_solve with every workspace buffer carved from a file-scope device array.
//
// For callers that cannot allocate device memory during a call (serving loops that budget memory up front,
// harnesses that forbid allocation).  Each GPU the library runs on holds its own copy of `scratch`, from the
// first context on that GPU until the process ends; its device address is looked up once per device, with
// that device current, when the context is created, and host code only ever passes that address (the
// array's name is a host-side stand-in, not a device pointer).  The solve then runs exactly as
// qp::solve does, with three differences that keep it from allocating: no tile autotuning (tuned or default
// tiles), no per-product timing events, and a BF16 stage buffer that may not grow.  Calls on one GPU share
// its scratch, so calls that overlap on one GPU (two streams, two threads, two contexts) race.
#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "aux.hpp"
#include "solver.hpp"

namespace qp {
namespace {

constexpr size_t kScratchBytes = size_t(QPINV_NOALLOC_SCRATCH_BYTES);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, void*> g_addr;  // device -> device address of that device's `scratch`

size_t align256(size_t b) { return (b + 255) / 256 * 256; }
int64_t round8(int64_t x) { return (x + 7) / 8 * 8; }

// bytes of a workspace matrix (ws_mat: ld padded to 8, plane stride padded to 8, four planes)
size_t mat_bytes(int64_t rows, int64_t cols, int dtype) {
  const int64_t ld = round8(std::max<int64_t>(cols, 1));
  const int64_t ps = round8(std::max<int64_t>(rows, 1) * ld);
  return align256(std::max<size_t>(256, (size_t)(4 * ps) * (dtype == QPINV_F64 ? 8 : 4)));
}

// Restores the context's allocating mode however the solve ends.
struct ArenaScope {
  Ctx& c;
  ArenaScope(Ctx& cx, void* base) : c(cx) {
    c.ws.begin_arena(base, kScratchBytes);
    c.no_alloc = true;
    c.scratch.no_grow = true;
  }
  ~ArenaScope() {
    c.ws.end_arena();
    c.no_alloc = false;
    c.scratch.no_grow = false;
  }
};

}  // namespace

void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_addr.find(device);
  if (it != g_addr.end()) return it->second;
  int cur = -1;
  QP_HIP(hipGetDevice(&cur));
  if (cur != device) throw Error(QPINV_EHIP, "no-allocation scratch: device " + std::to_string(device) + " is not current");
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(QPINV_EHIP, std::string("no-allocation scratch: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
  }
  g_addr[device] = p;
  return p;
}

// Every workspace request a solve can make, at its largest: per storage type of the precision phases the
// chain's 8 side-by-side buffers, 2 saved residuals, 4 iterates, 3 iterate-shaped temporaries, the
// residual-based and E1 outputs, E1's side product and a converted copy of A; the FP64 candidate check
// (iterate, X A, output, FP64 A); the refined FP64 finish (8 FP32 and 2 FP64 side-by-side, 2 FP32
// iterate-shaped); the Penrose projection; the zero result; the norm and power-iteration work vectors.
size_t noalloc_workspace_bound(int64_t m, int64_t n, int side, int precision, int out_dtype) {
  if (side == QPINV_SIDE_AUTO) side = (m > n) ? QPINV_SIDE_LEFT : QPINV_SIDE_RIGHT;
  const int64_t sd = side == QPINV_SIDE_LEFT ? n : m;
  const bool f32 = precision != QPINV_PREC_F64, f64 = precision != QPINV_PREC_F32;
  const bool finish = precision == QPINV_PREC_F32_F64FINISH || precision == QPINV_PREC_MIXED;
  size_t b = 0;
  for (int dt : {QPINV_F32, QPINV_F64}) {
    if ((dt == QPINV_F32 && !f32) || (dt == QPINV_F64 && !f64)) continue;
    b += 10 * mat_bytes(sd, sd, dt) + 8 * mat_bytes(n, m, dt) + 2 * mat_bytes(m, n, dt) +
         std::max(mat_bytes(n, n, dt), mat_bytes(m, m, dt));
  }
  b += 2 * mat_bytes(n, m, QPINV_F64) + mat_bytes(n, n, QPINV_F64) + mat_bytes(m, n, QPINV_F64);
  if (finish) b += 8 * mat_bytes(sd, sd, QPINV_F32) + 2 * mat_bytes(sd, sd, QPINV_F64) + 2 * mat_bytes(n, m, QPINV_F32);
  // the Penrose projection (FP64 copy, X A, A X, their adjoints, the first product, output, the update after it)
  b += 4 * mat_bytes(n, m, QPINV_F64) + 2 * mat_bytes(n, n, QPINV_F64) + 2 * mat_bytes(m, m, QPINV_F64);
  b += 32768;  // the one-launch path's parameter block (<= 20 KB), per-item sums (8 KB) and result record
  b += mat_bytes(n, m, out_dtype);
  b += align256(8 * (size_t)std::max(norms_work_doubles(m, n), norms_work_doubles(n, m)));
  b += align256(8 * (size_t)std::max(power_work_doubles(m, n), power_work_doubles(sd, sd)));
  return b;
}

int solve_noalloc(Ctx& c, int method, int order, const qpinv_qmat* A, int scaling, double alpha_or_mu, double tol,
                  int max_iter, int stop, int precision, qpinv_qmat* X, qpinv_info* info, hipStream_t s) {
  validate(A, "A");
  validate(X, "X");
  if (precision < QPINV_PREC_F64 || precision > QPINV_PREC_MIXED) throw Error(QPINV_EINVAL, "bad precision");
  const size_t need = noalloc_workspace_bound(A->rows, A->cols, c.opt.side, precision, X->dtype);
  if (need > kScratchBytes)
    throw Error(QPINV_EINVAL, "allocation-free solve: a " + std::to_string(A->rows) + " x " + std::to_string(A->cols) +
                                  " solve may need " + std::to_string(need) + " bytes of workspace, above the " +
                                  std::to_string(kScratchBytes) + "-byte no-allocation scratch");
  void* base = noalloc_scratch(c.device);
  ArenaScope scope(c, base);
  return solve(c, method, order, A, scaling, alpha_or_mu, tol, max_iter, stop, precision, X, info, s);
}

}  // namespace qp

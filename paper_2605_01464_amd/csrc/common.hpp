// Shared device/host definitions of the qpinv library (quaternion pseudoinverse on gfx950).
//
// Storage: a quaternion matrix A = A_s + A_x i + A_y j + A_z k (Section 2) is four real planes
// in one allocation, plane p at data + p * ps, row-major with row stride ld (elements).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <stdexcept>
#include <string>

namespace qp {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// A device view of one quaternion matrix (element type given by the user of the view).
struct QView {
  void* p = nullptr;
  int64_t rows = 0, cols = 0, ld = 0, ps = 0;
};

template <class T>
struct QV {
  T* p;
  int64_t ld, ps;
};

template <class T>
inline QV<T> qv(const QView& v) {
  return QV<T>{static_cast<T*>(v.p), v.ld, v.ps};
}

// Library error carried from the C++ layers to the C ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

}  // namespace qp

#define QP_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::qp::Error(-5, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

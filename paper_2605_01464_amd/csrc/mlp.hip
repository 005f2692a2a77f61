// Scaling network (learned alpha) kernels and state.
#include "mlp.hpp"

namespace qp {

struct MlpState {};

void mlp_free(Ctx* c) {
  if (c && c->mlp) {
    delete c->mlp;
    c->mlp = nullptr;
  }
}

}  // namespace qp

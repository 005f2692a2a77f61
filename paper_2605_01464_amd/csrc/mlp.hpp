// Scaling network (learned alpha): state owned by a context.
#pragma once

#include "solver.hpp"

namespace qp {

// Release the network state of a context (no-op when none was created).
void mlp_free(Ctx* c);

}  // namespace qp

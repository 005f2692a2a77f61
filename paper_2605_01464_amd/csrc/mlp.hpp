// Learned initial scaling: network state, training, inference and labels (host interface).
#pragma once

#include "solver.hpp"

namespace qp {

void mlp_free(Ctx* c);
int mlp_num_params();
// (Re)initialise the weights (Xavier-uniform from a SplitMix64 stream) and the Adam state.
void mlp_init(Ctx& c, uint64_t seed);
// Standardisation statistics of the ten network inputs over `count` raw feature rows (device).
void mlp_fit_normalization(Ctx& c, const double* raw, int count, hipStream_t s);
// One Adam step on the minibatch rows idx[0..batch) of (raw, target); with grad_out the gradient is
// written there instead and the weights stay.  Returns the minibatch loss.
double mlp_train_step(Ctx& c, const double* raw, const double* target, const int* idx, int batch, double lr,
                      float* grad_out, hipStream_t s);
// mu = exp(network(raw row)) for `count` rows (device arrays).
void mlp_predict(Ctx& c, const double* raw, int count, double* mu, hipStream_t s);
bool mlp_ready(Ctx& c);
// parameters followed by the standardisation (mean[10], std[10])
int mlp_get(Ctx& c, float* host, int n);
void mlp_set(Ctx& c, const float* host, int n);
void spectral_labels(Ctx& c, int method, int order, const double* spectra, const int* offsets, int count,
                     const double* s1sq_est, double tol, int max_iter, int ngrid, double mu_lo, double mu_hi,
                     double mu_target, double* mu_out, int* j_best, int* j_classical, hipStream_t s);

}  // namespace qp

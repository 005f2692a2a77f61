// Learned initial scaling: a 10 -> 64 -> 64 -> 1 tanh network predicting y = log(mu), with
// mu = alpha * sigma1_est^2 for X_0 = alpha A^H.  Training (forward, backpropagation, Adam), inference,
// input standardisation and the labels (iteration-count-minimising mu from a matrix's spectrum) all
// run in the kernels below.
//
// Network inputs: ten scale-invariant transforms of the raw features
//   raw = (s1sq, s1sq_prev, fro, norm1, norminf, m, n):
//   log m, log n, log(min/max), log(fro^2/s1sq), log(norm1 norminf/s1sq), log(norm1/norminf),
//   log(fro^2/(s1sq min)), s1sq_prev/s1sq, log(norm1/sqrt(m s1sq)), log(norminf/sqrt(n s1sq)).
// Parameters, one flat FP32 vector: W1 (10 x 64), b1 (64), W2 (64 x 64), b2 (64), W3 (64), b3.
#include <cmath>
#include <cstring>
#include <vector>

#include "mlp.hpp"

namespace qp {

constexpr int MF = 10, MH = 64;
constexpr int OW1 = 0, OB1 = OW1 + MF * MH, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH, OB3 = OW3 + MH;
constexpr int NPARAM = OB3 + 1;
constexpr int MAXB = 1024;  // largest training minibatch

struct MlpState {
  float* p = nullptr;     // parameters
  float* m = nullptr;     // Adam first moments
  float* v = nullptr;     // Adam second moments
  float* norm = nullptr;  // mean[10], std[10]
  float* act = nullptr;   // activations of one minibatch
  double* loss = nullptr; // device loss of the last step
  int step = 0;
  bool has_norm = false;
};

__device__ __forceinline__ void transform_raw(const double* r, float* f) {
  const double s1 = r[0], s1p = r[1], fro = r[2], n1 = r[3], ni = r[4], m = r[5], n = r[6];
  const double mn = fmin(m, n), mx = fmax(m, n);
  f[0] = (float)log(m);
  f[1] = (float)log(n);
  f[2] = (float)log(mn / mx);
  f[3] = (float)log(fro * fro / s1);
  f[4] = (float)log(n1 * ni / s1);
  f[5] = (float)log(n1 / ni);
  f[6] = (float)log(fro * fro / (s1 * mn));
  f[7] = (float)(s1p / s1);
  f[8] = (float)log(n1 / sqrt(m * s1));
  f[9] = (float)log(ni / sqrt(n * s1));
}

// ------------------------------------------------------------------------------------------------
// standardisation statistics (one workgroup, fixed-order sums)
// ------------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) norm_fit_kernel(const double* __restrict__ raw, int count, float* __restrict__ norm) {
  __shared__ double s1[256][MF], s2[256][MF];
  double a[MF], b[MF];
  for (int k = 0; k < MF; ++k) a[k] = b[k] = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) {
    float f[MF];
    transform_raw(raw + 7 * (int64_t)i, f);
    for (int k = 0; k < MF; ++k) {
      a[k] += f[k];
      b[k] += (double)f[k] * f[k];
    }
  }
  for (int k = 0; k < MF; ++k) {
    s1[threadIdx.x][k] = a[k];
    s2[threadIdx.x][k] = b[k];
  }
  __syncthreads();
  if (threadIdx.x < MF) {
    const int k = threadIdx.x;
    double sa = 0.0, sb = 0.0;
    for (int t = 0; t < 256; ++t) {
      sa += s1[t][k];
      sb += s2[t][k];
    }
    const double mean = sa / count;
    const double var = fmax(sb / count - mean * mean, 0.0);
    norm[k] = (float)mean;
    norm[MF + k] = (float)fmax(sqrt(var), 1e-6);
  }
}

// ------------------------------------------------------------------------------------------------
// one training step (or one gradient) on a minibatch: single workgroup, phases separated by barriers,
// every gradient entry summed over the batch in a fixed order
// ------------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) train_kernel(float* __restrict__ P, float* __restrict__ Mo, float* __restrict__ Vo,
                                                     const float* __restrict__ norm, const double* __restrict__ raw,
                                                     const double* __restrict__ target, const int* __restrict__ idx, int B,
                                                     float* __restrict__ act, int mode, float lr, int step,
                                                     float* __restrict__ grad_out, double* __restrict__ loss_out) {
  // act layout: Z[B][F], H1[B][H], H2[B][H], dy[B], D2[B][H], D1[B][H]
  float* Z = act;
  float* H1 = Z + MAXB * MF;
  float* H2 = H1 + MAXB * MH;
  float* dy = H2 + MAXB * MH;
  float* D2 = dy + MAXB;
  float* D1 = D2 + MAXB * MH;
  __shared__ double red[1024];
  const int tid = threadIdx.x, nt = blockDim.x;

  for (int b = tid; b < B; b += nt) {
    const int s = idx ? idx[b] : b;
    float f[MF];
    transform_raw(raw + 7 * (int64_t)s, f);
    for (int k = 0; k < MF; ++k) Z[b * MF + k] = (f[k] - norm[k]) / norm[MF + k];
  }
  __syncthreads();
  for (int e = tid; e < B * MH; e += nt) {
    const int b = e / MH, k = e % MH;
    float a = P[OB1 + k];
    for (int f = 0; f < MF; ++f) a += Z[b * MF + f] * P[OW1 + f * MH + k];
    H1[e] = tanhf(a);
  }
  __syncthreads();
  for (int e = tid; e < B * MH; e += nt) {
    const int b = e / MH, j = e % MH;
    float a = P[OB2 + j];
    for (int k = 0; k < MH; ++k) a += H1[b * MH + k] * P[OW2 + k * MH + j];
    H2[e] = tanhf(a);
  }
  __syncthreads();
  double lsum = 0.0;
  for (int b = tid; b < B; b += nt) {
    const int s = idx ? idx[b] : b;
    float y = P[OB3];
    for (int j = 0; j < MH; ++j) y += H2[b * MH + j] * P[OW3 + j];
    const float r = y - (float)target[s];
    dy[b] = 2.0f * r / (float)B;
    lsum += (double)r * r;
  }
  red[tid] = lsum;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0 && loss_out) loss_out[0] = red[0] / B;
  for (int e = tid; e < B * MH; e += nt) {
    const int b = e / MH, j = e % MH;
    const float h = H2[e];
    D2[e] = dy[b] * P[OW3 + j] * (1.0f - h * h);
  }
  __syncthreads();
  for (int e = tid; e < B * MH; e += nt) {
    const int b = e / MH, k = e % MH;
    float a = 0.f;
    for (int j = 0; j < MH; ++j) a += D2[b * MH + j] * P[OW2 + k * MH + j];
    const float h = H1[e];
    D1[e] = a * (1.0f - h * h);
  }
  __syncthreads();
  // gradient of every parameter: a fixed-order sum over the batch
  for (int q = tid; q < NPARAM; q += nt) {
    float g = 0.f;
    if (q < OB1) {
      const int f = q / MH, k = q % MH;
      for (int b = 0; b < B; ++b) g += Z[b * MF + f] * D1[b * MH + k];
    } else if (q < OW2) {
      const int k = q - OB1;
      for (int b = 0; b < B; ++b) g += D1[b * MH + k];
    } else if (q < OB2) {
      const int k = (q - OW2) / MH, j = (q - OW2) % MH;
      for (int b = 0; b < B; ++b) g += H1[b * MH + k] * D2[b * MH + j];
    } else if (q < OW3) {
      const int j = q - OB2;
      for (int b = 0; b < B; ++b) g += D2[b * MH + j];
    } else if (q < OB3) {
      const int j = q - OW3;
      for (int b = 0; b < B; ++b) g += H2[b * MH + j] * dy[b];
    } else {
      for (int b = 0; b < B; ++b) g += dy[b];
    }
    if (mode == 1) {
      grad_out[q] = g;
    } else {
      // Adam (Kingma & Ba): beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected
      const float m = 0.9f * Mo[q] + 0.1f * g;
      const float v = 0.999f * Vo[q] + 0.001f * g * g;
      Mo[q] = m;
      Vo[q] = v;
      const float mh = m / (1.0f - powf(0.9f, (float)step));
      const float vh = v / (1.0f - powf(0.999f, (float)step));
      P[q] -= lr * mh / (sqrtf(vh) + 1e-8f);
    }
  }
}

// y = log mu for `count` raw feature rows; mu = exp(y)
// Inference, one 64-lane wave per sample: lane k forms hidden unit k of each layer (its sums run over the
// layer's inputs in index order), and the output is the wave's sum of tanh(layer 2) * w3 plus the bias.
// A single solve thus waits for two short layers of parallel loads instead of one thread's 4.7k.
__global__ void __launch_bounds__(64) predict_kernel(const float* __restrict__ P, const float* __restrict__ norm,
                                                     const double* __restrict__ raw, int count, double* __restrict__ mu) {
  static_assert(MH == 64, "one lane per hidden unit");
  const int b = blockIdx.x, k = threadIdx.x;
  if (b >= count) return;
  __shared__ float h1s[MH];
  float f[MF];
  transform_raw(raw + 7 * (int64_t)b, f);
  for (int q = 0; q < MF; ++q) f[q] = (f[q] - norm[q]) / norm[MF + q];
  float a = P[OB1 + k];
  for (int q = 0; q < MF; ++q) a += f[q] * P[OW1 + q * MH + k];
  h1s[k] = tanhf(a);
  __syncthreads();
  float a2 = P[OB2 + k];
  for (int q = 0; q < MH; ++q) a2 += h1s[q] * P[OW2 + q * MH + k];
  float t = tanhf(a2) * P[OW3 + k];
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
  if (k == 0) mu[b] = exp((double)(P[OB3] + t));
}

// ------------------------------------------------------------------------------------------------
// labels: for each matrix (one workgroup) and grid point g (one thread), the iteration count J(alpha)
// to E1_rel <= tol in exact arithmetic from the spectrum: rho_i = 1 - alpha s_i^2, rho <- g(rho) per
// update, E1_rel^2 = sum s_i^2 rho_i^2 / sum s_i^2 (the iterates stay V diag U^H; Theorem 1's proof).
// Then the grid's argmin set, its longest contiguous run, and the point of that run nearest mu_target
// (the runs of high-order methods extend to the top of the admissible interval; a point near its top
// end is inside the run whenever the run is wide and still inside it when the run is narrow).
// ------------------------------------------------------------------------------------------------
constexpr int MAXJ = 64;

__device__ __forceinline__ double scalar_map(int method, int order, int qa, int qnu, double r) {
  switch (method) {
    case 0: return r * r;  // NS
    case 1: {              // hyperpower order p
      double o = 1.0;
      for (int k = 0; k < order; ++k) o *= r;
      return o;
    }
    case 2: {  // QSAI: r^10
      const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
      return r8 * r2;
    }
    case 3: {  // QHPI19: r^19
      const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4, r16 = r8 * r8;
      return r16 * r2 * r;
    }
    default: {  // QRAPID(N): 4^-a (3 + r)^a r^nu
      double o = 1.0, t = 0.25 * (3.0 + r);
      for (int k = 0; k < qa; ++k) o *= t;
      for (int k = 0; k < qnu; ++k) o *= r;
      return o;
    }
  }
}

__global__ void __launch_bounds__(256) labels_kernel(const double* __restrict__ spectra, const int* __restrict__ offsets,
                                                     const double* __restrict__ s1sq_est, int method, int order, int qa,
                                                     int qnu, double tol, int max_iter, int ngrid, double mu_lo, double mu_hi,
                                                     double mu_target, double* __restrict__ mu_out, int* __restrict__ j_best,
                                                     int* __restrict__ j_classical) {
  __shared__ int J[256];
  const int b = blockIdx.x, g = threadIdx.x;
  const double* s = spectra + offsets[b];
  const int r = offsets[b + 1] - offsets[b];
  double smax2 = 0.0, den = 0.0;
  for (int i = 0; i < r; ++i) {
    smax2 = fmax(smax2, s[i] * s[i]);
    den += s[i] * s[i];
  }
  const int lim = max_iter < MAXJ ? max_iter : MAXJ;
  // grid point g: mu_g geometric in [mu_lo, mu_hi] relative to the exact sigma_1^2; thread ngrid is the
  // classical alpha = 1 / sigma1_est^2
  double alpha;
  if (g < ngrid)
    alpha = mu_lo * pow(mu_hi / mu_lo, (double)g / (double)(ngrid - 1)) / smax2;
  else
    alpha = 1.0 / s1sq_est[b];
  int jb = lim + 1;
  if (g <= ngrid) {
    double acc[MAXJ];
    for (int j = 0; j < lim; ++j) acc[j] = 0.0;
    for (int i = 0; i < r; ++i) {
      const double w = s[i] * s[i];
      double rho = 1.0 - alpha * w;
      for (int j = 0; j < lim; ++j) {
        rho = scalar_map(method, order, qa, qnu, rho);
        if (!isfinite(rho) || fabs(rho) > 1e150) rho = 1e150;
        acc[j] += w * rho * rho;
      }
    }
    for (int j = 0; j < lim; ++j)
      if (sqrt(acc[j] / den) <= tol) {
        jb = j + 1;
        break;
      }
  }
  J[g] = jb;
  __syncthreads();
  if (g == 0) {
    int best = lim + 1;
    for (int k = 0; k < ngrid; ++k) best = min(best, J[k]);
    int run0 = -1, runlen = 0, cur0 = -1, curlen = 0;
    for (int k = 0; k < ngrid; ++k) {
      if (J[k] == best) {
        if (curlen == 0) cur0 = k;
        ++curlen;
        if (curlen > runlen) {
          runlen = curlen;
          run0 = cur0;
        }
      } else {
        curlen = 0;
      }
    }
    // the point of the run [run0, run0 + runlen - 1] nearest mu_target
    const double mu_a = mu_lo * pow(mu_hi / mu_lo, (double)run0 / (double)(ngrid - 1));
    const double mu_b = mu_lo * pow(mu_hi / mu_lo, (double)(run0 + runlen - 1) / (double)(ngrid - 1));
    const double mu_exact = fmin(fmax(mu_target, mu_a), mu_b);
    const double alpha_star = mu_exact / smax2;
    mu_out[b] = alpha_star * s1sq_est[b];
    j_best[b] = best;
    j_classical[b] = J[ngrid];
  }
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
static MlpState& state(Ctx& c) {
  if (!c.mlp) {
    c.mlp = new MlpState();
    MlpState& s = *c.mlp;
    QP_HIP(hipMalloc(&s.p, sizeof(float) * NPARAM));
    QP_HIP(hipMalloc(&s.m, sizeof(float) * NPARAM));
    QP_HIP(hipMalloc(&s.v, sizeof(float) * NPARAM));
    QP_HIP(hipMalloc(&s.norm, sizeof(float) * 2 * MF));
    QP_HIP(hipMalloc(&s.act, sizeof(float) * (MAXB * MF + 4 * MAXB * MH + MAXB)));
    QP_HIP(hipMalloc(&s.loss, sizeof(double)));
  }
  return *c.mlp;
}

void mlp_free(Ctx* c) {
  if (c && c->mlp) {
    MlpState& s = *c->mlp;
    for (void* p : {(void*)s.p, (void*)s.m, (void*)s.v, (void*)s.norm, (void*)s.act, (void*)s.loss})
      if (p) (void)hipFree(p);
    delete c->mlp;
    c->mlp = nullptr;
  }
}

int mlp_num_params() { return NPARAM; }

void mlp_init(Ctx& c, uint64_t seed) {
  MlpState& s = state(c);
  std::vector<float> h(NPARAM, 0.f);
  auto uni = [&](uint64_t k) {  // SplitMix64 counter stream -> [-1, 1)
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-52 - 1.0;
  };
  auto xavier = [&](int off, int fan_in, int fan_out, int count) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));
    for (int k = 0; k < count; ++k) h[off + k] = (float)(a * uni(off + k));
  };
  xavier(OW1, MF, MH, MF * MH);
  xavier(OW2, MH, MH, MH * MH);
  xavier(OW3, MH, 1, MH);
  QP_HIP(hipMemcpy(s.p, h.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  std::vector<float> z(NPARAM, 0.f);
  QP_HIP(hipMemcpy(s.m, z.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  QP_HIP(hipMemcpy(s.v, z.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  std::vector<float> nrm(2 * MF, 0.f);
  for (int k = 0; k < MF; ++k) nrm[MF + k] = 1.f;
  QP_HIP(hipMemcpy(s.norm, nrm.data(), sizeof(float) * 2 * MF, hipMemcpyHostToDevice));
  s.step = 0;
  s.has_norm = false;
}

void mlp_fit_normalization(Ctx& c, const double* raw, int count, hipStream_t st) {
  if (count < 1) throw Error(-1, "normalisation needs at least one sample");
  MlpState& s = state(c);
  hipLaunchKernelGGL(norm_fit_kernel, dim3(1), dim3(256), 0, st, raw, count, s.norm);
  QP_HIP(hipGetLastError());
  s.has_norm = true;
}

double mlp_train_step(Ctx& c, const double* raw, const double* target, const int* idx, int batch, double lr,
                      float* grad_out, hipStream_t st) {
  if (batch < 1 || batch > MAXB) throw Error(-1, "minibatch size must be in [1, 1024]");
  MlpState& s = state(c);
  const int mode = grad_out ? 1 : 0;
  if (!mode) ++s.step;
  hipLaunchKernelGGL(train_kernel, dim3(1), dim3(1024), 0, st, s.p, s.m, s.v, s.norm, raw, target, idx, batch, s.act, mode,
                     (float)lr, s.step, grad_out, s.loss);
  QP_HIP(hipGetLastError());
  double loss = 0.0;
  QP_HIP(hipMemcpyAsync(c.hsc, s.loss, sizeof(double), hipMemcpyDeviceToHost, st));
  QP_HIP(hipStreamSynchronize(st));
  loss = c.hsc[0];
  return loss;
}

void mlp_predict(Ctx& c, const double* raw, int count, double* mu, hipStream_t st) {
  MlpState& s = state(c);
  if (count <= 0) return;
  hipLaunchKernelGGL(predict_kernel, dim3(count), dim3(64), 0, st, s.p, s.norm, raw, count, mu);
  QP_HIP(hipGetLastError());
}

bool mlp_ready(Ctx& c) { return c.mlp && c.mlp->has_norm; }

int mlp_get(Ctx& c, float* host, int n) {
  MlpState& s = state(c);
  const int need = NPARAM + 2 * MF;
  if (!host || n < need) return need;
  QP_HIP(hipMemcpy(host, s.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
  QP_HIP(hipMemcpy(host + NPARAM, s.norm, sizeof(float) * 2 * MF, hipMemcpyDeviceToHost));
  return need;
}

void mlp_set(Ctx& c, const float* host, int n) {
  MlpState& s = state(c);
  const int need = NPARAM + 2 * MF;
  if (!host || n != need) throw Error(-1, "parameter vector has the wrong length");
  QP_HIP(hipMemcpy(s.p, host, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  QP_HIP(hipMemcpy(s.norm, host + NPARAM, sizeof(float) * 2 * MF, hipMemcpyHostToDevice));
  std::vector<float> z(NPARAM, 0.f);
  QP_HIP(hipMemcpy(s.m, z.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  QP_HIP(hipMemcpy(s.v, z.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  s.step = 0;
  s.has_norm = true;
}

void spectral_labels(Ctx& c, int method, int order, const double* spectra, const int* offsets, int count,
                     const double* s1sq_est, double tol, int max_iter, int ngrid, double mu_lo, double mu_hi,
                     double mu_target, double* mu_out, int* j_best, int* j_classical, hipStream_t st) {
  (void)c;
  if (count <= 0) return;
  if (ngrid < 2 || ngrid > 255) throw Error(-1, "label grid must have 2..255 points");
  if (!(mu_lo > 0.0) || !(mu_hi > mu_lo) || !(mu_hi < 2.0)) throw Error(-1, "label grid must lie in (0, 2)");
  if (!(mu_target > 0.0) || !(mu_target < 2.0)) throw Error(-1, "label target must lie in (0, 2)");
  int qa = 0, qnu = 0;
  int m = 3;
  switch (method) {
    case QPINV_NS: m = 0; break;
    case QPINV_HPI: m = 1; break;
    case QPINV_QSAI: m = 2; break;
    case QPINV_QHPI19: m = 3; break;
    default: {
      m = 4;
      auto fib = [](int k) {
        long a = 0, b = 1;
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
      qa = (int)fib(order + 2);
      qnu = (int)(11 * fib(order - 1) + 7 * fib(order - 2) + 1);
    }
  }
  hipLaunchKernelGGL(labels_kernel, dim3(count), dim3(256), 0, st, spectra, offsets, s1sq_est, m, order, qa, qnu, tol,
                     max_iter, ngrid, mu_lo, mu_hi, mu_target, mu_out, j_best, j_classical);
  QP_HIP(hipGetLastError());
}

}  // namespace qp

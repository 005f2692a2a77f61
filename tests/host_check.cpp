// Host-only checks of the library's host logic, built with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_host_sanitizers.py): the stop-rule controller on scripted and random per-update scalars, and
// the tune-cache text format (round trips, malformed and randomly mutated files).  Prints "host check ok"
// and exits 0 when every check holds; the sanitizers abort the run on the first memory or UB error.
#include <cmath>
#include <cstdio>
#include <limits>
#include <random>
#include <string>

#include "controller.hpp"
#include "tunecache.hpp"

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

using namespace qp;

static void controller_scripted() {
  {
    StopController c(STOP_DX_ABS, 1e-10);
    CHECK(c.update(1, 1.0, 2.0, -1.0) == D_CONTINUE);
    CHECK(c.update(2, 1e-12, 2.0, -1.0) == D_TOL);
  }
  {
    StopController c(STOP_DX_REL, 1e-9);
    CHECK(c.update(1, 1e-3, 2.0, -1.0) == D_CONTINUE);
    CHECK(c.update(2, 2e-9, 2.0, -1.0) == D_TOL);  // 2e-9 <= 1e-9 * 2
  }
  {
    StopController c(STOP_E1_REL, 1e-12);
    CHECK(c.update(1, 1.0, 1.0, 1e-9) == D_CONTINUE);
    CHECK(c.update(2, 1.0, 1.0, 1e-13) == D_TOL);
    CHECK(c.update(3, 1.0, 1.0, std::nan("")) == D_DIVERGED);
  }
  {
    StopController c(STOP_GUARDED, 1e-8);
    CHECK(c.update(1, 1.0, 1.0, -1.0) == D_NEWMIN);
    CHECK(c.update(2, std::numeric_limits<double>::infinity(), 1.0, -1.0) == D_DIVERGED);
  }
  {
    // fall, a floor at update 5, a rise at update 6
    const double rel[] = {0.9, 0.7, 0.2, 1e-3, 1e-5, 4e-5};
    StopController c(STOP_GUARDED, 1e-8);
    int last = -1;
    for (int j = 0; j < 6; ++j) last = c.update(j + 1, rel[j], 1.0, -1.0);
    CHECK(last == D_RISE);
    CHECK(c.best_j == 5);
  }
  {
    // a zero iterate norm gives d = 0: stop by tolerance, no division
    StopController c(STOP_GUARDED, 1e-8);
    CHECK(c.update(1, 0.5, 0.0, -1.0) == D_TOL);
  }
}

// Random sequences, including zeros, huge and non-finite values: every decision is a valid code, the rise
// rule only fires after a drop below half the running maximum, and a non-finite input is divergence.
static void controller_random(std::mt19937_64& rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  const double specials[] = {0.0, 1e-300, 1e300, std::numeric_limits<double>::infinity(), std::nan(""),
                             -1.0, std::numeric_limits<double>::denorm_min()};
  for (int trial = 0; trial < 20000; ++trial) {
    const int rule = (int)(rng() % 4);
    StopController c(rule, std::pow(10.0, -16.0 * u(rng)));
    for (int j = 1; j <= 40; ++j) {
      double d = std::pow(10.0, -20.0 * u(rng)), x = std::pow(10.0, 10.0 * u(rng) - 5.0), e = u(rng);
      if (rng() % 16 == 0) d = specials[rng() % 7];
      if (rng() % 16 == 0) x = specials[rng() % 7];
      if (rng() % 16 == 0) e = specials[rng() % 7];
      const double dmax0 = c.dmax, dprev0 = c.dprev;
      const int dec = c.update(j, d, x, e);
      CHECK(dec >= D_CONTINUE && dec <= D_NEWMIN);
      if (!std::isfinite(d) || !std::isfinite(x)) CHECK(dec == D_DIVERGED);
      if (dec == D_RISE) CHECK(rule == STOP_GUARDED && dprev0 >= 0.0 && dprev0 < 0.5 * dmax0);
      if (dec == D_TOL || dec == D_RISE || dec == D_DIVERGED) break;
    }
  }
}

static TuneFile sample_file(std::mt19937_64& rng) {
  TuneFile f;
  f.device = "gfx950:sramecc+:xnack-:256cu";
  const int ng = (int)(rng() % 6), nb = (int)(rng() % 4);
  for (int i = 0; i < ng; ++i)
    f.gemm.emplace_back((int)(rng() % 4), 1 + (int64_t)(rng() % 100000), 1 + (int64_t)(rng() % 100000),
                        1 + (int64_t)(rng() % 100000), "cfg_" + std::to_string(rng() % 50));
  for (int i = 0; i < nb; ++i) {
    std::vector<int64_t> sig(1 + rng() % 40);
    for (auto& v : sig) v = (int64_t)(rng() % 1000000) - 500000;
    f.batched.emplace_back(sig, "batched_" + std::to_string(rng() % 10));
  }
  return f;
}

static void tune_cache(std::mt19937_64& rng) {
  // round trips
  for (int trial = 0; trial < 500; ++trial) {
    const TuneFile f = sample_file(rng);
    TuneFile g;
    std::string err;
    CHECK(tune_parse(tune_format(f), g, err));
    CHECK(g.device == f.device && g.gemm == f.gemm && g.batched == f.batched);
  }
  // integer tokens at and past the int64 limits
  int64_t v = 0;
  CHECK(tune_int("9223372036854775807", v) && v == INT64_MAX);
  CHECK(tune_int("-9223372036854775808", v) && v == INT64_MIN);
  CHECK(!tune_int("9223372036854775808", v));
  CHECK(!tune_int("-9223372036854775809", v));
  CHECK(!tune_int("99999999999999999999999", v));
  CHECK(!tune_int("-", v) && !tune_int("", v) && !tune_int("1e3", v) && !tune_int("0x10", v));
  // malformed files are refused
  const char* bad[] = {
      "",
      "gemm 0 1 1 1 x\n",
      "qpinv-tune 2 dev\n",
      "qpinv-tune 1\n",
      "qpinv-tune 1 dev\ngemm 0 1 1 x\n",
      "qpinv-tune 1 dev\ngemm 4 1 1 1 x\n",
      "qpinv-tune 1 dev\ngemm 0 0 1 1 x\n",
      "qpinv-tune 1 dev\ngemm 0 1 1 1 x extra\n",
      "qpinv-tune 1 dev\nbatched x 3 1 2\n",
      "qpinv-tune 1 dev\nbatched x 0\n",
      "qpinv-tune 1 dev\nbatched x -1\n",
      "qpinv-tune 1 dev\nbatched x 9223372036854775807 1\n",
      "qpinv-tune 1 dev\nbatched x 2 1 y\n",
      "qpinv-tune 1 dev\nother 1\n",
  };
  for (const char* t : bad) {
    TuneFile g;
    std::string err;
    CHECK(!tune_parse(t, g, err) && !err.empty());
  }
  TuneFile g;
  std::string err;
  CHECK(tune_parse("\n  qpinv-tune 1 dev  \n\n gemm 1 2 3 4 name \n", g, err) && g.gemm.size() == 1);
  // random mutations of valid files: the parser accepts or refuses, without memory or UB errors
  const std::string alphabet = "0123456789 -+\nabgqx";
  for (int trial = 0; trial < 3000; ++trial) {
    std::string t = tune_format(sample_file(rng));
    const int edits = 1 + (int)(rng() % 6);
    for (int k = 0; k < edits && !t.empty(); ++k) {
      const size_t at = rng() % t.size();
      switch (rng() % 3) {
        case 0: t[at] = alphabet[rng() % alphabet.size()]; break;
        case 1: t.erase(at, 1 + rng() % 8); break;
        default: t.insert(at, std::string(1 + rng() % 4, alphabet[rng() % alphabet.size()])); break;
      }
    }
    TuneFile h;
    std::string e2;
    const bool ok = tune_parse(t, h, e2);
    CHECK(ok || !e2.empty());
  }
}

int main() {
  std::mt19937_64 rng(20260512);
  controller_scripted();
  controller_random(rng);
  tune_cache(rng);
  if (failures) {
    std::fprintf(stderr, "host check: %d failures\n", failures);
    return 1;
  }
  std::printf("host check ok\n");
  return 0;
}

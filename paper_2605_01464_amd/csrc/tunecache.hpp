// Persisted tile choices: the tuned product and batched-solver configurations of a context, as text.
//
//   qpinv-tune 1 <device>
//   gemm <product precision> <M> <N> <K> <configuration name>
//   batched <configuration name> <count> <count signature values>
//
// Configurations are stored by name, so a library whose tables changed skips the entries it no longer
// knows; the device token (architecture name and compute-unit count, no spaces) lets the loader refuse a
// file written on other hardware.  Host code only (no GPU use), also built on its own for the host
// sanitizer check.
#pragma once

#include <cstdint>
#include <sstream>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

namespace qp {

struct TuneFile {
  std::string device;
  std::vector<std::tuple<int, int64_t, int64_t, int64_t, std::string>> gemm;  // (prec, M, N, K, name)
  std::vector<std::pair<std::vector<int64_t>, std::string>> batched;          // (signature, name)
};

constexpr int kTuneVersion = 1;
constexpr int64_t kTuneMaxSignature = 1 << 20;  // values in one batched signature

inline std::string tune_format(const TuneFile& f) {
  std::ostringstream o;
  o << "qpinv-tune " << kTuneVersion << ' ' << f.device << '\n';
  for (const auto& g : f.gemm)
    o << "gemm " << std::get<0>(g) << ' ' << std::get<1>(g) << ' ' << std::get<2>(g) << ' ' << std::get<3>(g) << ' '
      << std::get<4>(g) << '\n';
  for (const auto& b : f.batched) {
    o << "batched " << b.second << ' ' << b.first.size();
    for (int64_t v : b.first) o << ' ' << v;
    o << '\n';
  }
  return o.str();
}

// One decimal integer token (optional sign, digits only, within int64).
inline bool tune_int(const std::string& t, int64_t& v) {
  if (t.empty() || t.size() > 20) return false;
  size_t i = (t[0] == '-' || t[0] == '+') ? 1 : 0;
  if (i == t.size()) return false;
  const bool neg = t[0] == '-';
  uint64_t acc = 0;
  for (; i < t.size(); ++i) {
    if (t[i] < '0' || t[i] > '9') return false;
    const uint64_t d = (uint64_t)(t[i] - '0');
    if (acc > (UINT64_C(9223372036854775808) - d) / 10) return false;
    acc = acc * 10 + d;
  }
  if (!neg && acc > (uint64_t)INT64_MAX) return false;
  v = neg ? (acc == UINT64_C(9223372036854775808) ? INT64_MIN : -(int64_t)acc) : (int64_t)acc;
  return true;
}

// Parses a whole file into f.  On a malformed file returns false with a message in err and leaves f
// partly filled (the caller applies nothing then).  Blank lines are ignored.
inline bool tune_parse(const std::string& text, TuneFile& f, std::string& err) {
  std::istringstream in(text);
  std::string line;
  int lineno = 0;
  bool header = false;
  auto fail = [&](const char* what) {
    err = "tune cache line " + std::to_string(lineno) + ": " + what;
    return false;
  };
  while (std::getline(in, line)) {
    ++lineno;
    std::istringstream ls(line);
    std::vector<std::string> tok;
    for (std::string t; ls >> t;) tok.push_back(t);
    if (tok.empty()) continue;
    if (!header) {
      int64_t ver = 0;
      if (tok.size() != 3 || tok[0] != "qpinv-tune" || !tune_int(tok[1], ver)) return fail("bad header");
      if (ver != kTuneVersion) return fail("unknown version");
      f.device = tok[2];
      header = true;
      continue;
    }
    if (tok[0] == "gemm") {
      int64_t p = 0, M = 0, N = 0, K = 0;
      if (tok.size() != 6 || !tune_int(tok[1], p) || !tune_int(tok[2], M) || !tune_int(tok[3], N) ||
          !tune_int(tok[4], K))
        return fail("bad gemm entry");
      if (p < 0 || p > 3 || M < 1 || N < 1 || K < 1) return fail("gemm entry out of range");
      f.gemm.emplace_back((int)p, M, N, K, tok[5]);
    } else if (tok[0] == "batched") {
      int64_t n = 0;
      if (tok.size() < 3 || !tune_int(tok[2], n)) return fail("bad batched entry");
      if (n < 1 || n > kTuneMaxSignature || (int64_t)tok.size() != 3 + n) return fail("bad batched signature length");
      std::vector<int64_t> sig((size_t)n);
      for (int64_t i = 0; i < n; ++i)
        if (!tune_int(tok[(size_t)(3 + i)], sig[(size_t)i])) return fail("bad batched signature value");
      f.batched.emplace_back(std::move(sig), tok[1]);
    } else {
      return fail("unknown entry");
    }
  }
  if (!header) {
    err = "tune cache: no header";
    return false;
  }
  return true;
}

}  // namespace qp

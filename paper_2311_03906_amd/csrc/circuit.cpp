// Circuit text parser and channel thresholds.
//
// Noise channels are the Pauli-fault symbols of Section 3.1: an X (Y, Z)
// error with probability p, one-qubit depolarizing with p/3 per non-identity
// Pauli, two-qubit depolarizing with p/15 per non-identity Pauli.  Each is
// sampled from one 32-bit draw u by integer thresholds
// T_k = floor(k * p * 2^32 / m), computed exactly from the decimal literal.
#include <cctype>
#include <cstring>
#include <map>
#include <sstream>

#include "sp_internal.hpp"

namespace sp {
namespace {

using u128 = unsigned __int128;

// Decimal literal -> (numerator, 10^k).  Grammar: digits [. digits] [e[+-]digits].
bool decimal_to_ratio(const std::string& s, u128& num, u128& den) {
  size_t i = 0, n = s.size();
  u128 mant = 0;
  int sig = 0, frac_digits = 0;
  bool dot = false, digits = false;
  for (; i < n; ++i) {
    char ch = s[i];
    if (ch >= '0' && ch <= '9') {
      digits = true;
      if (mant != 0 || ch != '0') {
        if (++sig > 19) return false;
      }
      mant = mant * 10u + (u128)(ch - '0');
      if (dot) ++frac_digits;
    } else if (ch == '.' && !dot) {
      dot = true;
    } else {
      break;
    }
  }
  if (!digits) return false;
  int exp10 = 0;
  if (i < n && (s[i] == 'e' || s[i] == 'E')) {
    ++i;
    bool neg = false;
    if (i < n && (s[i] == '+' || s[i] == '-')) neg = s[i++] == '-';
    if (i >= n || !std::isdigit((unsigned char)s[i])) return false;
    for (; i < n && std::isdigit((unsigned char)s[i]); ++i) {
      exp10 = exp10 * 10 + (s[i] - '0');
      if (exp10 > 60) return false;
    }
    if (neg) exp10 = -exp10;
  }
  if (i != n) return false;
  int e = exp10 - frac_digits;
  den = 1;
  if (e >= 0) {
    while (e-- > 0) {
      mant *= 10u;
      if (mant >> 100) return false;
    }
  } else {
    if (e < -30) return false;
    while (e++ < 0) den *= 10u;
  }
  num = mant;
  return true;
}

Channel make_channel(uint32_t kind, uint32_t m, const std::string& ptext) {
  u128 num = 0, den = 1;
  if (!decimal_to_ratio(ptext, num, den)) throw Error(SP_E_PARSE, "bad probability literal '" + ptext + "'");
  if (num > den) throw Error(SP_E_PARSE, "probability " + ptext + " exceeds 1");
  Channel ch;
  ch.kind = kind;
  ch.m = m;
  ch.ptext = ptext;
  for (uint32_t k = 1; k <= m; ++k) ch.T[k] = (uint64_t)((((u128)k * num) << 32) / (den * (u128)m));
  return ch;
}

struct NameInfo {
  OpKind kind;
  bool noise;
  uint32_t chan_kind;
  uint32_t m;
};

const std::map<std::string, NameInfo>& names() {
  static const std::map<std::string, NameInfo> tbl = {
      {"H", {OpKind::H, false, 0, 0}},
      {"S", {OpKind::S, false, 0, 0}},
      {"X", {OpKind::X, false, 0, 0}},
      {"Y", {OpKind::Y, false, 0, 0}},
      {"Z", {OpKind::Z, false, 0, 0}},
      {"CX", {OpKind::CX, false, 0, 0}},
      {"CNOT", {OpKind::CX, false, 0, 0}},
      {"M", {OpKind::M, false, 0, 0}},
      {"R", {OpKind::R, false, 0, 0}},
      {"MR", {OpKind::MR, false, 0, 0}},
      {"TICK", {OpKind::TICK, false, 0, 0}},
      {"X_ERROR", {OpKind::XERR, true, CH_XERR, 1}},
      {"Y_ERROR", {OpKind::YERR, true, CH_YERR, 1}},
      {"Z_ERROR", {OpKind::ZERR, true, CH_ZERR, 1}},
      {"DEPOLARIZE1", {OpKind::DEP1, true, CH_DEP1, 3}},
      {"DEPOLARIZE2", {OpKind::DEP2, true, CH_DEP2, 15}},
  };
  return tbl;
}

}  // namespace

sp_circuit* parse_circuit(const char* text, size_t len) {
  auto* c = new sp_circuit();
  try {
    c->channels.push_back(make_channel(CH_RANDBIT, 1, "0.5"));
    std::map<std::pair<uint32_t, std::string>, int32_t> chan_index;
    std::string all(text, len);
    std::istringstream lines(all);
    std::string line;
    int lineno = 0;
    uint64_t n_locs = 0, n_meas = 0;
    uint32_t max_q = 0;
    bool any_q = false;
    while (std::getline(lines, line)) {
      ++lineno;
      auto hash = line.find('#');
      if (hash != std::string::npos) line.resize(hash);
      std::istringstream toks(line);
      std::string head;
      if (!(toks >> head)) continue;
      const std::string where = "line " + std::to_string(lineno) + ": ";
      std::string name = head, ptext;
      auto lp = head.find('(');
      if (lp != std::string::npos) {
        if (head.back() != ')' || head.size() < lp + 3)
          throw Error(SP_E_PARSE, where + "malformed '" + head + "'");
        name = head.substr(0, lp);
        ptext = head.substr(lp + 1, head.size() - lp - 2);
      }
      auto it = names().find(name);
      if (it == names().end()) throw Error(SP_E_UNSUPPORTED, where + "unsupported instruction '" + name + "'");
      const NameInfo& ni = it->second;
      if (ni.noise != (lp != std::string::npos))
        throw Error(SP_E_PARSE, where + (ni.noise ? "missing probability for '" : "unexpected argument for '") + name + "'");
      Op op;
      op.kind = ni.kind;
      if (ni.noise) {
        auto key = std::make_pair(ni.chan_kind, ptext);
        auto ci = chan_index.find(key);
        if (ci == chan_index.end()) {
          Channel ch;
          try {
            ch = make_channel(ni.chan_kind, ni.m, ptext);
          } catch (const Error& e) {
            throw Error(e.code, where + e.what());
          }
          c->channels.push_back(ch);
          ci = chan_index.emplace(key, (int32_t)c->channels.size() - 1).first;
        }
        op.chan = ci->second;
      }
      std::string t;
      while (toks >> t) {
        if (t.empty() || t.size() > 9) throw Error(SP_E_PARSE, where + "bad target '" + t + "'");
        for (char ch : t)
          if (!std::isdigit((unsigned char)ch)) throw Error(SP_E_PARSE, where + "bad target '" + t + "'");
        uint32_t q = (uint32_t)std::stoul(t);
        if (q > 1000000) throw Error(SP_E_PARSE, where + "qubit index too large");
        op.targets.push_back(q);
        if (!any_q || q > max_q) max_q = q;
        any_q = true;
      }
      if (op.kind == OpKind::TICK && !op.targets.empty()) throw Error(SP_E_PARSE, where + "TICK takes no targets");
      if (op.kind == OpKind::CX || op.kind == OpKind::DEP2) {
        if (op.targets.size() % 2) throw Error(SP_E_PARSE, where + "targets must come in pairs");
        for (size_t i = 0; i < op.targets.size(); i += 2)
          if (op.targets[i] == op.targets[i + 1]) throw Error(SP_E_PARSE, where + "pair acts twice on one qubit");
      }
      switch (op.kind) {
        case OpKind::XERR: case OpKind::YERR: case OpKind::ZERR: case OpKind::DEP1: case OpKind::R:
          n_locs += op.targets.size(); break;
        case OpKind::DEP2: n_locs += op.targets.size() / 2; break;
        case OpKind::M: case OpKind::MR:
          n_locs += op.targets.size();
          n_meas += op.targets.size();
          break;
        default: break;
      }
      if (n_locs >= (1ull << 32)) throw Error(SP_E_LIMIT, "more than 2^32 locations");
      c->ops.push_back(std::move(op));
    }
    c->n_qubits = any_q ? max_q + 1 : 0;
    c->n_locs = (uint32_t)n_locs;
    c->n_meas = (uint32_t)n_meas;
    return c;
  } catch (...) {
    delete c;
    throw;
  }
}

}  // namespace sp

// Circuit text parser and channel thresholds.
//
// Noise channels are the Pauli-fault symbols of Section 3.1: an X (Y, Z)
// error with probability p, one-qubit depolarizing with p/3 per non-identity
// Pauli, two-qubit depolarizing with p/15 per non-identity Pauli.  Each is
// sampled from one 32-bit draw u by integer thresholds
// T_k = floor(k * p * 2^32 / m), computed exactly from the decimal literal.
#include <algorithm>
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

// How an instruction takes its parenthesized argument.
enum ArgKind : uint8_t { ARG_NONE, ARG_PROB, ARG_IGNORED, ARG_INDEX };

struct NameInfo {
  OpKind kind;
  ArgKind arg;
  uint32_t chan_kind;
  uint32_t m;
};

const std::map<std::string, NameInfo>& names() {
  static const std::map<std::string, NameInfo> tbl = {
      {"H", {OpKind::H, ARG_NONE, 0, 0}},
      {"S", {OpKind::S, ARG_NONE, 0, 0}},
      {"X", {OpKind::X, ARG_NONE, 0, 0}},
      {"Y", {OpKind::Y, ARG_NONE, 0, 0}},
      {"Z", {OpKind::Z, ARG_NONE, 0, 0}},
      {"CX", {OpKind::CX, ARG_NONE, 0, 0}},
      {"CNOT", {OpKind::CX, ARG_NONE, 0, 0}},
      {"CY", {OpKind::FY, ARG_NONE, 0, 0}},
      {"CZ", {OpKind::FZ, ARG_NONE, 0, 0}},
      {"M", {OpKind::M, ARG_NONE, 0, 0}},
      {"R", {OpKind::R, ARG_NONE, 0, 0}},
      {"MR", {OpKind::MR, ARG_NONE, 0, 0}},
      {"TICK", {OpKind::TICK, ARG_NONE, 0, 0}},
      {"DETECTOR", {OpKind::DET, ARG_IGNORED, 0, 0}},
      {"OBSERVABLE_INCLUDE", {OpKind::OBS, ARG_INDEX, 0, 0}},
      {"X_ERROR", {OpKind::XERR, ARG_PROB, CH_XERR, 1}},
      {"Y_ERROR", {OpKind::YERR, ARG_PROB, CH_YERR, 1}},
      {"Z_ERROR", {OpKind::ZERR, ARG_PROB, CH_ZERR, 1}},
      {"DEPOLARIZE1", {OpKind::DEP1, ARG_PROB, CH_DEP1, 3}},
      {"DEPOLARIZE2", {OpKind::DEP2, ARG_PROB, CH_DEP2, 15}},
  };
  return tbl;
}

// A target: a qubit index, or a measurement record rec[-k] (k >= 1).
struct Target {
  bool rec;
  uint32_t v;   // qubit, or k
};

bool parse_uint(const std::string& t, uint32_t limit, uint32_t* v) {
  if (t.empty() || t.size() > 9) return false;
  for (char ch : t)
    if (!std::isdigit((unsigned char)ch)) return false;
  const unsigned long x = std::stoul(t);
  if (x > limit) return false;
  *v = (uint32_t)x;
  return true;
}

Target parse_target(const std::string& t, const std::string& where) {
  Target r{false, 0};
  if (t.compare(0, 5, "rec[-") == 0 && t.size() > 6 && t.back() == ']') {
    r.rec = true;
    if (!parse_uint(t.substr(5, t.size() - 6), 1u << 30, &r.v) || r.v == 0)
      throw Error(SP_E_PARSE, where + "bad record target '" + t + "'");
    return r;
  }
  if (!parse_uint(t, 1000000, &r.v)) throw Error(SP_E_PARSE, where + "bad target '" + t + "'");
  return r;
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
    uint64_t n_locs = 0, n_meas = 0, n_det = 0, n_obs = 0;
    uint32_t max_q = 0;
    bool any_q = false;
    auto use_qubit = [&](uint32_t q) {
      if (!any_q || q > max_q) max_q = q;
      any_q = true;
    };
    while (std::getline(lines, line)) {
      ++lineno;
      auto hash = line.find('#');
      if (hash != std::string::npos) line.resize(hash);
      const std::string where = "line " + std::to_string(lineno) + ": ";
      // Head: a name, optionally followed by "(argument)".
      size_t i = 0;
      while (i < line.size() && std::isspace((unsigned char)line[i])) ++i;
      if (i == line.size()) continue;
      size_t j = i;
      while (j < line.size() && (std::isalnum((unsigned char)line[j]) || line[j] == '_')) ++j;
      const std::string name = line.substr(i, j - i);
      std::string arg;
      bool has_arg = false;
      if (j < line.size() && line[j] == '(') {
        const size_t close = line.find(')', j);
        if (close == std::string::npos) throw Error(SP_E_PARSE, where + "unclosed '(' after '" + name + "'");
        arg = line.substr(j + 1, close - j - 1);
        has_arg = true;
        j = close + 1;
      }
      if (name.empty() || (j < line.size() && !std::isspace((unsigned char)line[j])))
        throw Error(SP_E_PARSE, where + "malformed instruction");
      auto it = names().find(name);
      if (it == names().end()) throw Error(SP_E_UNSUPPORTED, where + "unsupported instruction '" + name + "'");
      const NameInfo& ni = it->second;
      if (ni.arg == ARG_PROB && !has_arg) throw Error(SP_E_PARSE, where + "missing probability for '" + name + "'");
      if ((ni.arg == ARG_NONE) && has_arg) throw Error(SP_E_PARSE, where + "unexpected argument for '" + name + "'");
      if (ni.arg == ARG_INDEX && !has_arg) throw Error(SP_E_PARSE, where + "missing index for '" + name + "'");
      std::vector<Target> tg;
      {
        std::istringstream toks(line.substr(j));
        std::string t;
        while (toks >> t) tg.push_back(parse_target(t, where));
      }
      // Record targets -> absolute measurement indices.
      auto record = [&](const Target& t) -> uint32_t {
        if (!t.rec) throw Error(SP_E_PARSE, where + "'" + name + "' takes record targets rec[-k]");
        if (t.v > n_meas) throw Error(SP_E_PARSE, where + "rec[-" + std::to_string(t.v) + "] precedes the first measurement");
        return (uint32_t)(n_meas - t.v);
      };
      auto qubit = [&](const Target& t) -> uint32_t {
        if (t.rec) throw Error(SP_E_PARSE, where + "'" + name + "' takes qubit targets here");
        use_qubit(t.v);
        return t.v;
      };
      auto push = [&](Op&& op) { c->ops.push_back(std::move(op)); };

      if (ni.kind == OpKind::CX || ni.kind == OpKind::FY || ni.kind == OpKind::FZ) {
        // (control, target) pairs: qubit pairs are CNOTs (CX only), record
        // pairs are Paulis controlled by a measurement.
        if (tg.size() % 2) throw Error(SP_E_PARSE, where + "targets must come in pairs");
        const OpKind fk = ni.kind == OpKind::CX ? OpKind::FX : ni.kind;
        Op cur;
        cur.kind = OpKind::TICK;
        for (size_t k = 0; k < tg.size(); k += 2) {
          const bool fb = tg[k].rec;
          if (!fb && ni.kind != OpKind::CX)
            throw Error(SP_E_UNSUPPORTED, where + "quantum '" + name + "' is outside the gate set (H, S, CNOT)");
          const OpKind kind = fb ? fk : OpKind::CX;
          if (cur.kind != kind && !cur.targets.empty()) push(std::move(cur));
          if (cur.kind != kind || cur.targets.empty()) { cur = Op(); cur.kind = kind; }
          if (fb) {
            cur.targets.push_back(record(tg[k]));
            cur.targets.push_back(qubit(tg[k + 1]));
          } else {
            const uint32_t a = qubit(tg[k]), b = qubit(tg[k + 1]);
            if (a == b) throw Error(SP_E_PARSE, where + "pair acts twice on one qubit");
            cur.targets.push_back(a);
            cur.targets.push_back(b);
          }
        }
        if (!cur.targets.empty()) push(std::move(cur));
        continue;
      }
      Op op;
      op.kind = ni.kind;
      if (ni.kind == OpKind::DET) {
        for (const Target& t : tg) op.targets.push_back(record(t));
        ++n_det;
        push(std::move(op));
        continue;
      }
      if (ni.kind == OpKind::OBS) {
        uint32_t idx = 0;
        if (!parse_uint(arg, 1000000, &idx)) throw Error(SP_E_PARSE, where + "bad observable index '" + arg + "'");
        op.targets.push_back(idx);
        for (const Target& t : tg) op.targets.push_back(record(t));
        n_obs = std::max<uint64_t>(n_obs, (uint64_t)idx + 1);
        push(std::move(op));
        continue;
      }
      if (ni.arg == ARG_PROB) {
        auto key = std::make_pair(ni.chan_kind, arg);
        auto ci = chan_index.find(key);
        if (ci == chan_index.end()) {
          Channel ch;
          try {
            ch = make_channel(ni.chan_kind, ni.m, arg);
          } catch (const Error& e) {
            throw Error(e.code, where + e.what());
          }
          c->channels.push_back(ch);
          ci = chan_index.emplace(key, (int32_t)c->channels.size() - 1).first;
        }
        op.chan = ci->second;
      }
      for (const Target& t : tg) op.targets.push_back(qubit(t));
      if (op.kind == OpKind::TICK && !op.targets.empty()) throw Error(SP_E_PARSE, where + "TICK takes no targets");
      if (op.kind == OpKind::DEP2) {
        if (op.targets.size() % 2) throw Error(SP_E_PARSE, where + "targets must come in pairs");
        for (size_t k = 0; k < op.targets.size(); k += 2)
          if (op.targets[k] == op.targets[k + 1]) throw Error(SP_E_PARSE, where + "pair acts twice on one qubit");
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
      if (n_locs >= (1ull << 32) || n_meas >= (1ull << 31)) throw Error(SP_E_LIMIT, "more than 2^32 locations");
      push(std::move(op));
    }
    if (n_det >= (1ull << 31) || n_det + n_obs >= (1ull << 31)) throw Error(SP_E_LIMIT, "too many detectors");
    c->n_qubits = any_q ? max_q + 1 : 0;
    c->n_locs = (uint32_t)n_locs;
    c->n_meas = (uint32_t)n_meas;
    c->n_detectors = (uint32_t)n_det;
    c->n_observables = (uint32_t)n_obs;
    return c;
  } catch (...) {
    delete c;
    throw;
  }
}

// Circuit-level noise added to a circuit (the noise model P_C): a channel
// after every one-qubit gate (DEPOLARIZE1) and every CNOT pair
// (DEPOLARIZE2), X_ERROR before every M/MR and after every R/MR, and, at
// each TICK, DEPOLARIZE1 on every qubit that no gate, measurement, reset or
// controlled Pauli of the layer since the previous TICK touched.  A null or
// empty probability adds nothing.
sp_circuit* add_noise(const sp_circuit& in, const sp_noise& spec) {
  auto* c = new sp_circuit(in);
  try {
    std::map<std::pair<uint32_t, std::string>, int32_t> chan_index;
    for (size_t k = 1; k < c->channels.size(); ++k)
      chan_index.emplace(std::make_pair(c->channels[k].kind, c->channels[k].ptext), (int32_t)k);
    auto chan = [&](uint32_t kind, uint32_t m, const std::string& p) {
      auto key = std::make_pair(kind, p);
      auto it = chan_index.find(key);
      if (it != chan_index.end()) return it->second;
      c->channels.push_back(make_channel(kind, m, p));
      return chan_index.emplace(key, (int32_t)c->channels.size() - 1).first->second;
    };
    struct Chan {
      bool on;
      OpKind kind;
      int32_t idx;
    };
    auto make = [&](const char* p, OpKind kind, uint32_t ck, uint32_t m) {
      Chan r{p && *p, kind, -1};
      if (r.on) r.idx = chan(ck, m, p);
      return r;
    };
    const Chan g1 = make(spec.p_1q, OpKind::DEP1, CH_DEP1, 3), g2 = make(spec.p_2q, OpKind::DEP2, CH_DEP2, 15);
    const Chan meas = make(spec.p_meas, OpKind::XERR, CH_XERR, 1), reset = make(spec.p_reset, OpKind::XERR, CH_XERR, 1);
    const Chan idle = make(spec.p_idle, OpKind::DEP1, CH_DEP1, 3);

    std::vector<Op> ops;
    uint64_t n_locs = 0;
    std::vector<uint8_t> touched(c->n_qubits, 0);
    auto noise = [&](const Chan& ch, const std::vector<uint32_t>& targets) {
      if (!ch.on || targets.empty()) return;
      Op op;
      op.kind = ch.kind;
      op.chan = ch.idx;
      op.targets = targets;
      n_locs += ch.kind == OpKind::DEP2 ? targets.size() / 2 : targets.size();
      ops.push_back(std::move(op));
    };
    for (const Op& op : in.ops) {
      switch (op.kind) {
        case OpKind::H: case OpKind::S: case OpKind::X: case OpKind::Y: case OpKind::Z: case OpKind::CX:
          for (uint32_t q : op.targets) touched[q] = 1;
          ops.push_back(op);
          noise(op.kind == OpKind::CX ? g2 : g1, op.targets);
          break;
        case OpKind::M: case OpKind::MR: case OpKind::R:
          for (uint32_t q : op.targets) touched[q] = 1;
          if (op.kind != OpKind::R) noise(meas, op.targets);
          ops.push_back(op);
          n_locs += op.targets.size();
          if (op.kind != OpKind::M) noise(reset, op.targets);
          break;
        case OpKind::FX: case OpKind::FY: case OpKind::FZ:
          for (size_t k = 1; k < op.targets.size(); k += 2) touched[op.targets[k]] = 1;
          ops.push_back(op);
          break;
        case OpKind::TICK: {
          std::vector<uint32_t> idle_q;
          for (uint32_t q = 0; q < c->n_qubits; ++q)
            if (!touched[q]) idle_q.push_back(q);
          noise(idle, idle_q);
          std::fill(touched.begin(), touched.end(), 0);
          ops.push_back(op);
          break;
        }
        case OpKind::XERR: case OpKind::YERR: case OpKind::ZERR: case OpKind::DEP1:
          n_locs += op.targets.size();
          ops.push_back(op);
          break;
        case OpKind::DEP2:
          n_locs += op.targets.size() / 2;
          ops.push_back(op);
          break;
        default:
          ops.push_back(op);
          break;
      }
      if (n_locs >= (1ull << 32)) throw Error(SP_E_LIMIT, "more than 2^32 locations");
    }
    c->ops.swap(ops);
    c->n_locs = (uint32_t)n_locs;
    return c;
  } catch (...) {
    delete c;
    throw;
  }
}

}  // namespace sp

// Initialization of Algorithm 1: the A-G tableau with symbolic phases.
//
// Section 3.2.1 encodes a phase expression as a bit vector over the symbols
// s_0 (the constant 1), s_1 .. s_ns.  Section 3.2.2 extends the A-G tableau
// (Eq. 1) with one such vector per row (Eq. 3) and updates it with
//   Init-C  H/S/CNOT act on the X|Z columns as in A-G; the constant column
//           takes the phase change A-G would apply to r;
//   Init-P  a fault X^{s_j} (Z^{s_j}) adds s_j to the rows with z_a = 1
//           (x_a = 1), the Pauli-gate rules of Fact 1;
//   Init-M  measurements follow A-G's row operations, adding whole vectors
//           where A-G adds phase bits; a random outcome is a fresh symbol, a
//           determined one is the vector of the scratch row.
// By Fact 2 no branch depends on a phase, so this single pass serves every
// assignment of the symbols.
//
// Representation.  A phase vector is kept sparse: the constant bit plus the
// ascending list of symbol indices present.  Only stabilizer rows (and the
// scratch row) carry vectors: destabilizer phases are never added into a
// stabilizer or into the scratch row, so no outcome depends on them.
//
// Random measurement.  The new stabilizer row Z_a receives the fresh symbol
// and no other row does (the A-G random branch, and the bell example's
// printed tableau after M_1).  The sentence describing this case also speaks
// of applying an X^s at the measured qubit; that would flip every row with
// z_a = 1 and contradicts the printed example, so it is not followed.
//
// Reset R = measure without recording, then X^e with e the outcome's vector
// (the conditional-Pauli idea of the conclusion).  MR = M, then X^e.  A
// Pauli controlled by a recorded measurement k is P^{e_k} the same way.
//
// Outputs.  The rows of (M, c) are the recorded measurements' vectors, or
// (detector outputs) each detector's and observable's sum of them.
#include <algorithm>
#include <cstring>

#include "sp_internal.hpp"

namespace sp {
namespace {

using Phase = Expr;   // c: coefficient of s_0; v: ascending variable indices

// a <- a + b over GF(2)
void phase_add(Phase& a, const Phase& b, std::vector<uint32_t>& tmp) {
  a.c ^= b.c;
  if (b.v.empty()) return;
  if (a.v.empty()) {
    a.v = b.v;
    return;
  }
  tmp.clear();
  tmp.reserve(a.v.size() + b.v.size());
  size_t i = 0, j = 0;
  while (i < a.v.size() && j < b.v.size()) {
    if (a.v[i] < b.v[j]) tmp.push_back(a.v[i++]);
    else if (a.v[i] > b.v[j]) tmp.push_back(b.v[j++]);
    else { ++i; ++j; }
  }
  tmp.insert(tmp.end(), a.v.begin() + i, a.v.end());
  tmp.insert(tmp.end(), b.v.begin() + j, b.v.end());
  a.v.swap(tmp);
}

class SymTableau {
 public:
  explicit SymTableau(uint32_t n) : n_(n), nw_(n ? (n + 63) / 64 : 1) {
    x_.assign((size_t)(2 * n + 1) * nw_, 0);
    z_.assign((size_t)(2 * n + 1) * nw_, 0);
    ph_.resize(n + 1);  // stabilizers 0..n-1, scratch n
    for (uint32_t i = 0; i < n; ++i) {
      flip(xr(i), i);        // destabilizer i = X_i
      flip(zr(n + i), i);    // stabilizer i = Z_i
    }
  }

  // --- Init-C ---------------------------------------------------------
  void h(uint32_t a) {
    for (uint32_t i = 0; i < 2 * n_; ++i) {
      int x = bit(xr(i), a), z = bit(zr(i), a);
      if (i >= n_ && (x & z)) ph_[i - n_].c ^= 1;
      if (x != z) { flip(xr(i), a); flip(zr(i), a); }
    }
  }
  void s(uint32_t a) {
    for (uint32_t i = 0; i < 2 * n_; ++i) {
      int x = bit(xr(i), a), z = bit(zr(i), a);
      if (i >= n_ && (x & z)) ph_[i - n_].c ^= 1;
      if (x) flip(zr(i), a);
    }
  }
  void cx(uint32_t a, uint32_t b) {
    for (uint32_t i = 0; i < 2 * n_; ++i) {
      int xa = bit(xr(i), a), za = bit(zr(i), a), xb = bit(xr(i), b), zb = bit(zr(i), b);
      if (i >= n_ && (xa & zb & (xb ^ za ^ 1))) ph_[i - n_].c ^= 1;
      if (xa) flip(xr(i), b);
      if (zb) flip(zr(i), a);
    }
  }
  // Pauli gate X^px Z^pz with a constant exponent (Fact 1).
  void pauli_const(uint32_t a, int px, int pz) {
    for (uint32_t i = n_; i < 2 * n_; ++i)
      if ((px & bit(zr(i), a)) ^ (pz & bit(xr(i), a))) ph_[i - n_].c ^= 1;
  }
  // --- Init-P: X^{s_var} (px) or Z^{s_var} (pz) on qubit a ----------------
  // `var` is the newest variable, so appending keeps each list ascending.
  void pauli_var(uint32_t a, int px, int pz, uint32_t var) {
    for (uint32_t i = n_; i < 2 * n_; ++i)
      if ((px & bit(zr(i), a)) ^ (pz & bit(xr(i), a))) ph_[i - n_].v.push_back(var);
  }
  // X^(px e) Z^(pz e) with a vector exponent e: a reset after a
  // measurement with outcome e (X^e), or a Pauli controlled by a recorded
  // measurement (the conditional Paulis of the conclusion).  Like a fault,
  // it adds e to the rows it anticommutes with.
  void pauli_expr(uint32_t a, int px, int pz, const Phase& e) {
    for (uint32_t i = n_; i < 2 * n_; ++i)
      if ((px & bit(zr(i), a)) ^ (pz & bit(xr(i), a))) phase_add(ph_[i - n_], e, tmp_);
  }

  // --- Init-M ---------------------------------------------------------
  // Returns true (and sets out = {new_var}) for a random outcome.
  bool measure(uint32_t a, uint32_t new_var, Phase& out) {
    int64_t p = -1;
    const uint32_t w = a >> 6;
    const uint64_t m = 1ull << (a & 63);
    for (uint32_t i = n_; i < 2 * n_; ++i)
      if (xr(i)[w] & m) { p = i; break; }
    if (p >= 0) {
      for (uint32_t i = 0; i < 2 * n_; ++i) {
        if (i == (uint32_t)p || !(xr(i)[w] & m)) continue;
        if (i < n_) rowsum_xz(i, (uint32_t)p);
        else rowsum_sym(i, (uint32_t)p);
      }
      std::memcpy(xr((uint32_t)p - n_), xr((uint32_t)p), nw_ * 8);
      std::memcpy(zr((uint32_t)p - n_), zr((uint32_t)p), nw_ * 8);
      std::memset(xr((uint32_t)p), 0, nw_ * 8);
      std::memset(zr((uint32_t)p), 0, nw_ * 8);
      flip(zr((uint32_t)p), a);
      Phase& pp = ph_[(uint32_t)p - n_];
      pp.c = 0;
      pp.v.assign(1, new_var);
      out = pp;
      return true;
    }
    const uint32_t sc = 2 * n_;
    std::memset(xr(sc), 0, nw_ * 8);
    std::memset(zr(sc), 0, nw_ * 8);
    ph_[n_].c = 0;
    ph_[n_].v.clear();
    for (uint32_t i = 0; i < n_; ++i)
      if (xr(i)[w] & m) rowsum_sym(sc, n_ + i);
    out = ph_[n_];
    return false;
  }

 private:
  uint64_t* xr(uint32_t i) { return &x_[(size_t)i * nw_]; }
  uint64_t* zr(uint32_t i) { return &z_[(size_t)i * nw_]; }
  static int bit(const uint64_t* r, uint32_t j) { return (int)((r[j >> 6] >> (j & 63)) & 1u); }
  static void flip(uint64_t* r, uint32_t j) { r[j >> 6] ^= 1ull << (j & 63); }

  void rowsum_xz(uint32_t h, uint32_t i) {
    uint64_t *xh = xr(h), *zh = zr(h);
    const uint64_t *xi = xr(i), *zi = zr(i);
    for (uint32_t k = 0; k < nw_; ++k) { xh[k] ^= xi[k]; zh[k] ^= zi[k]; }
  }
  // Row h <- row i * row h (h, i stabilizer or scratch rows).  The product's
  // sign is (-1)^(r_h + r_i) times i^(sum g); with commuting rows the sum is
  // 0 or 2 mod 4, the latter flipping the constant.
  void rowsum_sym(uint32_t h, uint32_t i) {
    uint64_t *xh = xr(h), *zh = zr(h);
    const uint64_t *xi = xr(i), *zi = zr(i);
    int64_t g = 0;
    for (uint32_t k = 0; k < nw_; ++k) {
      const uint64_t a = xi[k], b = zi[k], c = xh[k], d = zh[k];
      // +1: X*Y, Y*Z, Z*X;  -1: X*Z, Y*X, Z*Y  (left factor from row i)
      const uint64_t plus = (a & ~b & c & d) | (a & b & ~c & d) | (~a & b & c & ~d);
      const uint64_t minus = (a & ~b & ~c & d) | (a & b & c & ~d) | (~a & b & c & d);
      g += __builtin_popcountll(plus) - __builtin_popcountll(minus);
      xh[k] = a ^ c;
      zh[k] = b ^ d;
    }
    Phase& ph = ph_[h - n_];
    if ((((g % 4) + 4) % 4) == 2) ph.c ^= 1;
    phase_add(ph, ph_[i - n_], tmp_);
  }

  uint32_t n_, nw_;
  std::vector<uint64_t> x_, z_;
  std::vector<Phase> ph_;
  std::vector<uint32_t> tmp_;
};

}  // namespace

sp_model* symbolize(const sp_circuit& c, int outputs) {
  SymTableau tab(c.n_qubits);
  std::vector<Phase> outcomes;
  outcomes.reserve(c.n_meas);
  std::vector<int32_t> loc_var0;
  loc_var0.reserve(c.n_locs);
  uint64_t n_vars = 0;
  uint32_t n_random = 0;
  auto take_vars = [&](uint32_t k) {
    uint64_t v = n_vars;
    n_vars += k;
    if (n_vars >= (1ull << 24)) throw Error(SP_E_LIMIT, "more than 2^24 variables");
    return v;
  };
  try {
    for (const Op& op : c.ops) {
      const auto& t = op.targets;
      switch (op.kind) {
        case OpKind::H: for (uint32_t q : t) tab.h(q); break;
        case OpKind::S: for (uint32_t q : t) tab.s(q); break;
        case OpKind::X: for (uint32_t q : t) tab.pauli_const(q, 1, 0); break;
        case OpKind::Y: for (uint32_t q : t) tab.pauli_const(q, 1, 1); break;
        case OpKind::Z: for (uint32_t q : t) tab.pauli_const(q, 0, 1); break;
        case OpKind::CX: for (size_t i = 0; i < t.size(); i += 2) tab.cx(t[i], t[i + 1]); break;
        case OpKind::TICK: case OpKind::DET: case OpKind::OBS: break;
        case OpKind::FX: case OpKind::FY: case OpKind::FZ: {
          const int px = op.kind != OpKind::FZ, pz = op.kind != OpKind::FX;
          for (size_t i = 0; i < t.size(); i += 2) {
            const Phase e = outcomes[t[i]];   // a copy: the tableau update may not alias it
            tab.pauli_expr(t[i + 1], px, pz, e);
          }
          break;
        }
        case OpKind::XERR: case OpKind::YERR: case OpKind::ZERR: {
          const int px = op.kind != OpKind::ZERR, pz = op.kind != OpKind::XERR;
          for (uint32_t q : t) {
            uint32_t v = (uint32_t)take_vars(1);
            loc_var0.push_back((int32_t)v);
            tab.pauli_var(q, px, pz, v);  // Y^s = X^s Z^s: rows with x xor z
          }
          break;
        }
        case OpKind::DEP1:
          for (uint32_t q : t) {
            uint32_t v = (uint32_t)take_vars(2);
            loc_var0.push_back((int32_t)v);
            tab.pauli_var(q, 1, 0, v);       // bit 0: X^{s}
            tab.pauli_var(q, 0, 1, v + 1);   // bit 1: Z^{s'}
          }
          break;
        case OpKind::DEP2:
          for (size_t i = 0; i < t.size(); i += 2) {
            uint32_t v = (uint32_t)take_vars(4);
            loc_var0.push_back((int32_t)v);
            tab.pauli_var(t[i], 1, 0, v);
            tab.pauli_var(t[i], 0, 1, v + 1);
            tab.pauli_var(t[i + 1], 1, 0, v + 2);
            tab.pauli_var(t[i + 1], 0, 1, v + 3);
          }
          break;
        case OpKind::M: case OpKind::R: case OpKind::MR:
          for (uint32_t q : t) {
            Phase e;
            bool rnd = tab.measure(q, (uint32_t)n_vars, e);
            if (rnd) {
              loc_var0.push_back((int32_t)take_vars(1));
              ++n_random;
            } else {
              loc_var0.push_back(-1);
            }
            if (op.kind != OpKind::R) outcomes.push_back(e);
            if (op.kind != OpKind::M) tab.pauli_expr(q, 1, 0, e);
          }
          break;
      }
    }
  } catch (const std::bad_alloc&) {
    throw Error(SP_E_NOMEM, "out of host memory in symbolize");
  }
  return assemble_model(c, outputs, std::move(loc_var0), (uint32_t)n_vars, n_random, outcomes);
}

sp_model* assemble_model(const sp_circuit& c, int outputs, std::vector<int32_t> loc_var0, uint32_t n_vars,
                         uint32_t n_random, const std::vector<Expr>& outcomes) {
  if (loc_var0.size() != c.n_locs || outcomes.size() != c.n_meas)
    throw Error(SP_E_INVALID, "inconsistent Initialization result");
  auto* mdl = new sp_model();
  try {
    mdl->n_qubits = c.n_qubits;
    mdl->outputs = outputs;
    mdl->n_locs = c.n_locs;
    mdl->channels = c.channels;
    mdl->n_vars = n_vars;
    mdl->n_random = n_random;
    mdl->loc_var0 = std::move(loc_var0);
    mdl->loc_kind.reserve(c.n_locs);
    mdl->loc_chan.reserve(c.n_locs);
    std::vector<Phase> dets, obs(c.n_observables);
    std::vector<uint32_t> tmp;
    auto loc = [&](uint8_t kind, int32_t chan) {
      const uint32_t l = (uint32_t)mdl->loc_kind.size();
      const int32_t v0 = mdl->loc_var0[l];
      mdl->loc_kind.push_back(kind);
      mdl->loc_chan.push_back(v0 < 0 ? -1 : chan);
      if (v0 >= 0)
        for (uint32_t b = 0; b < loc_bits(kind); ++b) {
          mdl->var_loc.push_back(l);
          mdl->var_bit.push_back((uint8_t)b);
        }
    };
    for (const Op& op : c.ops) {
      const auto& t = op.targets;
      switch (op.kind) {
        case OpKind::XERR: for (size_t i = 0; i < t.size(); ++i) loc(L_XERR, op.chan); break;
        case OpKind::YERR: for (size_t i = 0; i < t.size(); ++i) loc(L_YERR, op.chan); break;
        case OpKind::ZERR: for (size_t i = 0; i < t.size(); ++i) loc(L_ZERR, op.chan); break;
        case OpKind::DEP1: for (size_t i = 0; i < t.size(); ++i) loc(L_DEP1, op.chan); break;
        case OpKind::DEP2: for (size_t i = 0; i < t.size(); i += 2) loc(L_DEP2, op.chan); break;
        case OpKind::M: for (size_t i = 0; i < t.size(); ++i) loc(L_M, 0); break;
        case OpKind::R: for (size_t i = 0; i < t.size(); ++i) loc(L_R, 0); break;
        case OpKind::MR: for (size_t i = 0; i < t.size(); ++i) loc(L_MR, 0); break;
        case OpKind::DET: {
          Phase d;
          for (uint32_t k : t) phase_add(d, outcomes[k], tmp);
          dets.push_back(std::move(d));
          break;
        }
        case OpKind::OBS:
          for (size_t i = 1; i < t.size(); ++i) phase_add(obs[t[0]], outcomes[t[i]], tmp);
          break;
        default: break;
      }
    }
    if (mdl->var_loc.size() != n_vars) throw Error(SP_E_INVALID, "inconsistent variable count");

    // The output rows: recorded measurements, or detectors then observables.
    const std::vector<Phase>* rows = &outcomes;
    if (outputs == SP_OUT_DETECTORS) {
      for (Phase& o : obs) dets.push_back(std::move(o));
      rows = &dets;
    }
    mdl->n_meas = (uint32_t)rows->size();

    // M as column lists, rows ascending; c as bits.
    mdl->col_ptr.assign((size_t)n_vars + 1, 0);
    mdl->c_bits.assign((rows->size() + 63) / 64 + 1, 0);
    for (const Phase& p : *rows)
      for (uint32_t v : p.v) mdl->col_ptr[v + 1]++;
    for (uint64_t j = 0; j < n_vars; ++j) mdl->col_ptr[j + 1] += mdl->col_ptr[j];
    mdl->row_idx.resize(mdl->col_ptr[n_vars]);
    std::vector<uint32_t> fill(mdl->col_ptr.begin(), mdl->col_ptr.end() - 1);
    for (uint32_t k = 0; k < rows->size(); ++k) {
      for (uint32_t v : (*rows)[k].v) mdl->row_idx[fill[v]++] = k;
      if ((*rows)[k].c) mdl->c_bits[k >> 6] |= 1ull << (k & 63);
    }
    return mdl;
  } catch (const std::bad_alloc&) {
    delete mdl;
    throw Error(SP_E_NOMEM, "out of host memory in symbolize");
  } catch (...) {
    delete mdl;
    throw;
  }
}

}  // namespace sp

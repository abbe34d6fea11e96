// Internal host-side types of the sampler library.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/symphase.h"

namespace sp {

// Error carried to the C boundary as (code, message).
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// FX/FY/FZ: a Pauli on a qubit controlled by a recorded measurement (targets:
// pairs of absolute measurement index, qubit).  DET: a detector (targets:
// absolute measurement indices).  OBS: a contribution to an observable
// (targets: the observable index, then absolute measurement indices).
enum class OpKind : uint8_t { H, S, X, Y, Z, CX, M, R, MR, XERR, YERR, ZERR, DEP1, DEP2, TICK, FX, FY, FZ, DET, OBS };

// Channel kinds as seen by the sampling kernel.  RANDBIT is the fair coin of
// a random measurement (threshold 2^31).
enum ChanKind : uint32_t { CH_RANDBIT = 0, CH_XERR = 1, CH_YERR = 2, CH_ZERR = 3, CH_DEP1 = 4, CH_DEP2 = 5 };

struct Channel {
  uint32_t kind = 0;
  uint32_t m = 1;          // number of non-identity codes
  uint64_t T[16] = {0};    // T[1..m]; T[m] may equal 2^32 (p = 1)
  std::string ptext;
};

struct Op {
  OpKind kind;
  std::vector<uint32_t> targets;
  int32_t chan = -1;  // channel index for noise instructions
};

// Location kinds (program order numbering, see symphase.h).
enum LocKind : uint8_t { L_XERR = 1, L_YERR = 2, L_ZERR = 3, L_DEP1 = 4, L_DEP2 = 5, L_M = 6, L_R = 7, L_MR = 8 };

inline uint32_t loc_bits(uint8_t k) {
  switch (k) {
    case L_DEP1: return 2;
    case L_DEP2: return 4;
    default: return 1;
  }
}

}  // namespace sp

struct sp_circuit {
  uint32_t n_qubits = 0;
  uint32_t n_locs = 0;
  uint32_t n_meas = 0;
  uint32_t n_detectors = 0;
  uint32_t n_observables = 0;
  std::vector<sp::Op> ops;
  std::vector<sp::Channel> channels;  // channels[0] is the random-measurement coin
};

struct sp_model {
  // n_meas counts the output rows: recorded measurements, or detectors then
  // observables (outputs == SP_OUT_DETECTORS).
  uint32_t n_qubits = 0, n_meas = 0, n_locs = 0, n_vars = 0, n_random = 0;
  int outputs = 0;
  std::vector<sp::Channel> channels;
  // per location
  std::vector<uint8_t> loc_kind;
  std::vector<int32_t> loc_chan;   // channel index or -1 (determined measurement)
  std::vector<int32_t> loc_var0;   // first variable or -1
  // per variable
  std::vector<uint32_t> var_loc;
  std::vector<uint8_t> var_bit;
  // M as column lists (CSC), rows ascending; c as a bit vector
  std::vector<uint32_t> col_ptr;
  std::vector<uint32_t> row_idx;
  std::vector<uint64_t> c_bits;
};

namespace sp {
// A location the sampler draws for: a channel that can fire (T_m > 0) whose
// variables reach at least one output row.  Any other location cannot change
// an output, and since every draw is keyed by its own location, leaving it
// out changes no other draw.
inline bool loc_drawn(const sp_model& m, uint32_t l) {
  const int32_t ch = m.loc_chan[l];
  if (ch < 0 || m.channels[ch].T[m.channels[ch].m] == 0) return false;
  const uint32_t v0 = (uint32_t)m.loc_var0[l];
  return m.col_ptr[v0 + loc_bits(m.loc_kind[l])] > m.col_ptr[v0];
}

// A phase expression over GF(2): the constant bit plus the ascending list of
// variable indices present (variable j = symbol s_{j+1} of Section 3.2.1).
struct Expr {
  uint8_t c = 0;
  std::vector<uint32_t> v;
};

sp_circuit* parse_circuit(const char* text, size_t len);
// A copy of the circuit with the channels of a circuit-level noise model
// added (see sp_circuit_add_noise).
sp_circuit* add_noise(const sp_circuit& c, const sp_noise& noise);
sp_model* symbolize(const sp_circuit& c, int outputs);
// The model from one Initialization pass: loc_var0 per location (-1 for a
// determined measurement), the variable count, and the expression of every
// recorded measurement.  Builds the location table, the output rows
// (measurements, or detectors then observables) and (M, c) as column lists.
sp_model* assemble_model(const sp_circuit& c, int outputs, std::vector<int32_t> loc_var0, uint32_t n_vars,
                         uint32_t n_random, const std::vector<Expr>& outcomes);
}  // namespace sp

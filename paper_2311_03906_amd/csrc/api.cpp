// C ABI entry points for the host-side stages (parse, symbolize, exports).
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "sp_internal.hpp"

namespace sp {
thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
}  // namespace sp

using sp::set_error;

#define SP_GUARD_BEGIN try {
#define SP_GUARD_END                                                   \
  }                                                                    \
  catch (const sp::Error& e) { return set_error(e.code, e.what()); }   \
  catch (const std::bad_alloc&) { return set_error(SP_E_NOMEM, "out of host memory"); } \
  catch (const std::exception& e) { return set_error(SP_E_INVALID, e.what()); } \
  catch (...) { return set_error(SP_E_INVALID, "unknown error"); }

extern "C" {

const char* sp_last_error(void) { return sp::g_last_error.c_str(); }

int sp_circuit_parse(const char* text, size_t len, sp_circuit** out) {
  SP_GUARD_BEGIN
  if (!out) return set_error(SP_E_INVALID, "out is null");
  *out = nullptr;
  if (!text && len) return set_error(SP_E_INVALID, "text is null");
  *out = sp::parse_circuit(text ? text : "", len);
  return SP_OK;
  SP_GUARD_END
}

void sp_circuit_free(sp_circuit* c) { delete c; }

int sp_circuit_add_noise(const sp_circuit* c, const sp_noise* noise, sp_circuit** out) {
  SP_GUARD_BEGIN
  if (!out) return set_error(SP_E_INVALID, "out is null");
  *out = nullptr;
  if (!c || !noise) return set_error(SP_E_INVALID, "null argument");
  *out = sp::add_noise(*c, *noise);
  return SP_OK;
  SP_GUARD_END
}

int sp_circuit_counts(const sp_circuit* c, uint32_t* n_qubits, uint32_t* n_meas, uint32_t* n_detectors,
                      uint32_t* n_observables) {
  if (!c) return set_error(SP_E_INVALID, "null circuit");
  if (n_qubits) *n_qubits = c->n_qubits;
  if (n_meas) *n_meas = c->n_meas;
  if (n_detectors) *n_detectors = c->n_detectors;
  if (n_observables) *n_observables = c->n_observables;
  return SP_OK;
}

int sp_symbolize_outputs(const sp_circuit* c, int outputs, sp_model** out) {
  SP_GUARD_BEGIN
  if (!c || !out) return set_error(SP_E_INVALID, "null argument");
  *out = nullptr;
  if (outputs != SP_OUT_MEASUREMENTS && outputs != SP_OUT_DETECTORS)
    return set_error(SP_E_INVALID, "unknown outputs " + std::to_string(outputs));
  *out = sp::symbolize(*c, outputs);
  return SP_OK;
  SP_GUARD_END
}

int sp_symbolize(const sp_circuit* c, sp_model** out) { return sp_symbolize_outputs(c, SP_OUT_MEASUREMENTS, out); }

void sp_model_free(sp_model* m) { delete m; }

int sp_model_dims(const sp_model* m, sp_dims* d) {
  if (!m || !d) return set_error(SP_E_INVALID, "null argument");
  d->n_qubits = m->n_qubits;
  d->n_meas = m->n_meas;
  d->n_locs = m->n_locs;
  d->n_vars = m->n_vars;
  d->n_random_meas = m->n_random;
  uint32_t drawn = 0, blocks = 0;
  int64_t last_block = -1;
  for (uint32_t l = 0; l < m->n_locs; ++l) {
    if (sp::loc_drawn(*m, l)) {
      ++drawn;
      if ((int64_t)(l >> 2) != last_block) {
        ++blocks;
        last_block = l >> 2;
      }
    }
  }
  d->n_drawn = drawn;
  d->n_draw_blocks = blocks;
  d->reserved = 0;
  d->nnz = m->row_idx.size();
  return SP_OK;
}

int sp_model_expected_work(const sp_model* m, double* fired_per_word, double* entries_per_word) {
  if (!m) return set_error(SP_E_INVALID, "null model");
  double fired = 0, entries = 0;
  for (uint32_t l = 0; l < m->n_locs; ++l) {
    if (!sp::loc_drawn(*m, l)) continue;
    const sp::Channel& c = m->channels[m->loc_chan[l]];
    const double q = (double)c.T[c.m] / 4294967296.0;
    const double f = 1.0 - std::pow(1.0 - q, 64.0);
    fired += f;
    const uint32_t v0 = (uint32_t)m->loc_var0[l];
    const uint32_t nv = sp::loc_bits(m->loc_kind[l]);
    entries += f * (double)(m->col_ptr[v0 + nv] - m->col_ptr[v0]);
  }
  if (fired_per_word) *fired_per_word = fired;
  if (entries_per_word) *entries_per_word = entries;
  return SP_OK;
}

int sp_model_export_dense(const sp_model* m, uint64_t* M, size_t row_words, uint64_t* c) {
  if (!m || (!M && m->n_meas)) return set_error(SP_E_INVALID, "null argument");
  if (M) {
    if (row_words < (m->n_vars + 63) / 64) return set_error(SP_E_INVALID, "row_words too small");
    std::memset(M, 0, sizeof(uint64_t) * row_words * m->n_meas);
    for (uint32_t j = 0; j < m->n_vars; ++j)
      for (uint32_t i = m->col_ptr[j]; i < m->col_ptr[j + 1]; ++i)
        M[(size_t)m->row_idx[i] * row_words + (j >> 6)] |= 1ull << (j & 63);
  }
  if (c) std::memcpy(c, m->c_bits.data(), sizeof(uint64_t) * ((m->n_meas + 63) / 64));
  return SP_OK;
}

int sp_model_export_csc(const sp_model* m, uint32_t* col_ptr, uint32_t* row_idx) {
  if (!m || !col_ptr || (!row_idx && !m->row_idx.empty())) return set_error(SP_E_INVALID, "null argument");
  std::memcpy(col_ptr, m->col_ptr.data(), sizeof(uint32_t) * m->col_ptr.size());
  if (!m->row_idx.empty()) std::memcpy(row_idx, m->row_idx.data(), sizeof(uint32_t) * m->row_idx.size());
  return SP_OK;
}

int sp_model_export_vars(const sp_model* m, uint32_t* var_loc, uint8_t* var_bit) {
  if (!m || ((!var_loc || !var_bit) && m->n_vars)) return set_error(SP_E_INVALID, "null argument");
  if (m->n_vars) {
    std::memcpy(var_loc, m->var_loc.data(), sizeof(uint32_t) * m->n_vars);
    std::memcpy(var_bit, m->var_bit.data(), m->n_vars);
  }
  return SP_OK;
}

}  // extern "C"

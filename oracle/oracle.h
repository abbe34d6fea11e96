/*
 * oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain CPU reference for the sampling path: every shot is simulated from
 * scratch with the concrete Aaronson-Gottesman stabilizer tableau (the
 * improved tableau with destabilizers, paper Section 2.2, Eq. 1), with the
 * Pauli faults of that shot applied as the Pauli gates of Fact 1.  It shares
 * no code with the sampling library: its own circuit parser, its own
 * exact-decimal thresholds and its own Philox4x32-10.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.
 *
 * All functions return 0 on success and a negative value on error; the
 * message is available from oracle_last_error().
 */
#ifndef SYMPHASE_ORACLE_H
#define SYMPHASE_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_circuit oracle_circuit;

/* Location kinds, as reported by oracle_location_kinds(). */
enum {
  ORACLE_LOC_X_ERROR = 1,
  ORACLE_LOC_Y_ERROR = 2,
  ORACLE_LOC_Z_ERROR = 3,
  ORACLE_LOC_DEPOLARIZE1 = 4,
  ORACLE_LOC_DEPOLARIZE2 = 5,
  ORACLE_LOC_M = 6,
  ORACLE_LOC_R = 7,
  ORACLE_LOC_MR = 8
};

int oracle_parse(const char* text, size_t len, oracle_circuit** out);
void oracle_free(oracle_circuit* c);
/* n_qubits, number of locations, number of recorded measurements. */
int oracle_dims(const oracle_circuit* c, int* n_qubits, int* n_locs, int* n_meas);
/* kinds[l] for every location l (ORACLE_LOC_*). */
int oracle_location_kinds(const oracle_circuit* c, int* kinds);

/* One shot with explicit per-location codes (no random numbers):
 *   X/Y/Z_ERROR: code 1 applies the Pauli, 0 nothing;
 *   DEPOLARIZE1: code k in 0..3 applies X^(k&1) Z^(k>>1);
 *   DEPOLARIZE2: code k in 0..15 applies X^(bit0) Z^(bit1) on the first qubit
 *                and X^(bit2) Z^(bit3) on the second;
 *   M/R/MR:      bit 0 of the code is the outcome if the measurement is random
 *                (ignored when it is determined).
 * outcomes: n_meas bytes (0/1).  was_random (nullable): n_locs bytes, set to
 * 1 for measurement locations whose outcome was random.  If check_invariants
 * is nonzero the tableau commutation relations are verified after every
 * instruction (slow; for small circuits). */
int oracle_run_codes(const oracle_circuit* c, const uint8_t* codes, uint8_t* outcomes,
                     uint8_t* was_random, int check_invariants);

/* Philox4x32-10 block function: out = Philox(ctr, key). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* The draw of location l in shot `shot` under `seed`. */
uint32_t oracle_draw(uint64_t seed, uint64_t shot, uint64_t loc);
/* Thresholds T_1..T_m (as 64-bit, T_m may equal 2^32) for a channel whose
 * m non-identity outcomes each have probability p/m, p a decimal literal. */
int oracle_thresholds(const char* p_text, int m, uint64_t* T);
/* Per-location codes drawn for one shot (n_locs bytes). Measurement
 * locations get the random-outcome bit. */
int oracle_draw_codes(const oracle_circuit* c, uint64_t seed, uint64_t shot, uint8_t* codes);

/* Samples shots [first_shot, first_shot+shots) into the packed layout:
 * out[k*ld + w] bit b = outcome of measurement k in shot first_shot+64w+b.
 * Writes n_meas*ld words (bits past `shots` and words past the last one are
 * zero).  n_threads <= 0 means one per available core. */
int oracle_sample(const oracle_circuit* c, uint64_t seed, uint64_t first_shot, uint64_t shots,
                  uint64_t* out, size_t ld, int n_threads);
/* Outcomes of individual shots: outcomes[i*n_meas + k]. */
int oracle_sample_shots(const oracle_circuit* c, uint64_t seed, const uint64_t* shot_ids,
                        size_t n, uint8_t* outcomes, int n_threads);

/* Detector outputs.  outputs = 0: rows are the recorded measurements (as
 * above); outputs = 1: rows are the detectors in program order, then
 * observables 0, 1, ...; each is the XOR of the shot's outcomes it names. */
int oracle_output_dims(const oracle_circuit* c, int* n_detectors, int* n_observables);
int oracle_rows_from_outcomes(const oracle_circuit* c, int outputs, const uint8_t* outcomes, uint8_t* rows);
int oracle_sample_outputs(const oracle_circuit* c, int outputs, uint64_t seed, uint64_t first_shot, uint64_t shots,
                          uint64_t* out, size_t ld, int n_threads);
int oracle_sample_shots_outputs(const oracle_circuit* c, int outputs, uint64_t seed, const uint64_t* shot_ids,
                                size_t n, uint8_t* rows, int n_threads);

const char* oracle_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

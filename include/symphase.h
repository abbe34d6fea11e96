/*
 * symphase.h -- C ABI of the phase-symbolization sampler for AMD Instinct
 * MI355X (gfx950).
 *
 * The paper states the problem as: given a noisy stabilizer circuit C with a
 * noise model P_C and a sample count, return that many samples of all
 * measurements (Algorithm 1, its input/output lines).  Algorithm 1 splits it
 * into Initialization(C) -> m_1..m_nm and Sampling(n_smp, P_C, m_1..m_nm) ->
 * M_samples.  This library maps those to
 *
 *   sp_circuit_parse (+ sp_circuit_add_noise for a noise model P_C)
 *   sp_symbolize                      Initialization, on the host
 *                                     (Section 3.2.2: Init-C, Init-P, Init-M)
 *   sp_symbolize_device               the same Initialization on the GPU
 *   sp_model_upload                   make (M, c, P_C) resident on the GPU
 *   sp_sample                         Sampling, on the GPU (Section 3.2.3, Eq. 4)
 *   sp_sample_host                    the same Sampling on the host CPU
 *
 * Conventions
 *   - Every function returns SP_OK (0) or a negative SP_E_* code; the message
 *     is in sp_last_error() (thread-local, valid until the next call on the
 *     same thread).  No C++ exception crosses this boundary.  Arguments are
 *     validated before any device work is queued.
 *   - Handles (sp_circuit, sp_model, sp_dmodel) are owned by the library and
 *     released by the matching *_free function, which accepts NULL.
 *   - The library allocates no device memory.  The device model lives in a
 *     caller-provided device buffer; sample outputs are caller-provided device
 *     buffers.  (sp_sample_batch_static uses a fixed array in the library's
 *     device image instead of a work buffer.)  `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream); device work is queued on it asynchronously.
 *
 * Circuit text: one instruction per line, '#' comments.
 *   H S X Y Z <q...>            Clifford / Pauli gates
 *   CX <c t ...>                CNOT on (control, target) pairs
 *   M <q...>   R <q...>   MR <q...>   measure / reset / measure-then-reset (Z basis)
 *   X_ERROR(p) Y_ERROR(p) Z_ERROR(p) <q...>   Pauli fault with probability p
 *   DEPOLARIZE1(p) <q...>       X, Y, Z each with probability p/3
 *   DEPOLARIZE2(p) <a b ...>    each of the 15 non-identity two-qubit Paulis with p/15
 *   CX rec[-k] <q>  CY rec[-k] <q>  CZ rec[-k] <q>
 *                               X / Y / Z on q when the k-th most recent recorded
 *                               measurement was 1 (the conditional Paulis X^e, Y^e,
 *                               Z^e of the paper's conclusion; e is that
 *                               measurement's expression); several (rec, q)
 *                               pairs may follow, and CX may mix them with
 *                               CNOT pairs
 *   DETECTOR[(args)] rec[-k] ...          a detector: the XOR of the named records
 *                                         (args, e.g. coordinates, are ignored)
 *   OBSERVABLE_INCLUDE(i) rec[-k] ...     XORs the named records into observable i
 *   TICK
 * p is an exact decimal literal in [0, 1].  rec[-k] (k >= 1) names the k-th
 * most recent measurement recorded before the instruction.
 *
 * Locations, variables and draws (the sampling contract)
 *   - A location l is, in program order, each target of a one-qubit channel,
 *     each pair of DEPOLARIZE2, and each target of M, R and MR.
 *   - For shot index t (absolute: first_shot + i) and 64-bit seed,
 *       u(l) = Philox4x32-10(ctr = (l/4, t mod 2^32, t / 2^32, 0),
 *                            key = (seed mod 2^32, seed / 2^32))[l mod 4].
 *   - A channel whose m non-identity outcomes each have probability p/m
 *     (m = 1, 3, 15) has thresholds T_k = floor(k * p * 2^32 / m); it picks
 *     code k when T_{k-1} <= u < T_k (T_0 = 0), identity when u >= T_m.
 *     Code bits: X/Y/Z_ERROR fire on code 1; DEPOLARIZE1 code k is
 *     X^(bit0) Z^(bit1); DEPOLARIZE2 code k is X^(bit0) Z^(bit1) on the first
 *     qubit and X^(bit2) Z^(bit3) on the second.
 *   - A measurement whose outcome is random (Init-M, first case) takes the
 *     bit [u(l) < 2^31]; a determined one draws nothing.
 *   - A location on which no output row depends is not drawn at all; no
 *     output depends on its draw, and no other draw changes.
 *   - Variables (columns of M) are numbered in location order; a noise
 *     location owns one variable per code bit (bit order), a random
 *     measurement owns one, a determined measurement none.
 *
 * Output layout (M_samples of Eq. 4, packed 64 shots per word)
 *   out[k * ld_words + w], bit b (LSB = 0) = output row k in shot
 *   first_shot + 64 w + b.  Bits for shots >= `shots` are written as 0; words
 *   w >= ceil(shots/64) are not written.  Rows are the recorded measurements
 *   in program order (SP_OUT_MEASUREMENTS), or the detectors in program order
 *   followed by observables 0, 1, ... (SP_OUT_DETECTORS): each such row is the
 *   XOR of its records, so its expression is the XOR of their rows of (M, c).
 */
#ifndef SYMPHASE_H
#define SYMPHASE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SP_OK 0
#define SP_E_INVALID (-1)     /* bad argument (null pointer, size, alignment) */
#define SP_E_PARSE (-2)       /* malformed circuit text or probability */
#define SP_E_UNSUPPORTED (-3) /* instruction outside the stabilizer gate set */
#define SP_E_NOMEM (-4)       /* host allocation failed */
#define SP_E_DEVICE (-5)      /* HIP runtime error (message included) */
#define SP_E_LIMIT (-6)       /* a size exceeds what the kernels support */
#define SP_E_BUDGET (-7)      /* a server request can never fit, or its queue is full */
#define SP_E_TIMEOUT (-8)     /* a wait ended before the request finished */

typedef struct sp_circuit sp_circuit; /* parsed circuit (host) */
typedef struct sp_model sp_model;     /* (M, c) and the location table (host) */
typedef struct sp_dmodel sp_dmodel;   /* device-resident model */

typedef struct {
  uint32_t n_qubits;
  uint32_t n_meas;        /* output rows = rows of M (see SP_OUT_*) */
  uint32_t n_locs;        /* locations */
  uint32_t n_vars;        /* variables = columns of M (the constant excluded) */
  uint32_t n_random_meas; /* M/R/MR locations whose outcome is random */
  uint32_t n_drawn;       /* locations the sampler draws for: p > 0 or random, and
                             some output row depends on them */
  uint32_t n_draw_blocks; /* distinct l/4 over drawn locations = Philox blocks per shot */
  uint32_t reserved;
  uint64_t nnz;           /* nonzero entries of M (the constant column excluded) */
} sp_dims;

/* Evaluation path of the sampling kernel for out = M s + c (Eq. 4). */
enum {
  SP_PATH_AUTO = 0,   /* chosen from the column density of M */
  SP_PATH_SPARSE = 1, /* per fired variable, XOR into the rows of its column list */
  SP_PATH_DENSE = 2   /* per fired variable, XOR into the rows set in its n_m-bit mask */
};

/* Output rows of a model. */
enum {
  SP_OUT_MEASUREMENTS = 0, /* every recorded measurement */
  SP_OUT_DETECTORS = 1     /* every detector, then every observable */
};

/* Parses circuit text (len bytes, need not be NUL-terminated).
 * Errors: SP_E_INVALID (null), SP_E_PARSE, SP_E_UNSUPPORTED. */
int sp_circuit_parse(const char* text, size_t len, sp_circuit** out);
void sp_circuit_free(sp_circuit* circuit);

/* A noise model P_C (Algorithm 1's input) as circuit-level channels, each
 * probability a decimal literal (thresholds are exact, as for channels in
 * the text), NULL or "" for none:
 *   p_1q     DEPOLARIZE1 after every target of H, S, X, Y, Z
 *   p_2q     DEPOLARIZE2 after every pair of CX
 *   p_meas   X_ERROR before every target of M and MR
 *   p_reset  X_ERROR after every target of R and MR
 *   p_idle   at every TICK, DEPOLARIZE1 on each qubit that no gate,
 *            measurement, reset or controlled Pauli touched since the
 *            previous TICK (qubits ascending); after the last TICK, none.
 * Each channel follows (or, for p_meas, precedes) its instruction, so
 * locations are numbered as if the channels were written in the text. */
typedef struct {
  const char* p_1q;
  const char* p_2q;
  const char* p_meas;
  const char* p_reset;
  const char* p_idle;
} sp_noise;

/* A new circuit: `circuit` with the noise model's channels added (the
 * channels already in the text stay).  *out is owned by the caller
 * (sp_circuit_free).  Errors: SP_E_INVALID (null), SP_E_PARSE (a
 * probability literal that is malformed or above 1), SP_E_LIMIT. */
int sp_circuit_add_noise(const sp_circuit* circuit, const sp_noise* noise, sp_circuit** out);

/* Counts of a parsed circuit (any pointer may be NULL): qubits, recorded
 * measurements, detectors, observables (1 + the largest index used). */
int sp_circuit_counts(const sp_circuit* circuit, uint32_t* n_qubits, uint32_t* n_meas, uint32_t* n_detectors,
                      uint32_t* n_observables);

/* Algorithm 1, Initialization: one forward pass of the tableau with symbolic
 * phases (Section 3.2.2; Init-C for H/S/CNOT, Init-P for each fault variable,
 * Init-M for measurements; reset is measure-then-conditional-X, the X
 * exponent being the outcome's expression).  The noise model P_C is the set
 * of channel instructions in the circuit.  Errors: SP_E_INVALID, SP_E_NOMEM,
 * SP_E_LIMIT. */
int sp_symbolize(const sp_circuit* circuit, sp_model** out);
/* The same pass with a choice of output rows (SP_OUT_*): with
 * SP_OUT_DETECTORS the rows of (M, c) are the detectors' and observables'
 * expressions, sums of measurement expressions.  Errors as sp_symbolize,
 * and SP_E_INVALID for an unknown `outputs`. */
int sp_symbolize_outputs(const sp_circuit* circuit, int outputs, sp_model** out);
void sp_model_free(sp_model* model);

/* Initialization (Section 3.2.2, Algorithm 1) on the GPU: the same pass as
 * sp_symbolize_outputs, and the same model, bit for bit, computed by one
 * 1024-thread workgroup on `stream` over a bit-packed tableau in the
 * caller's device work buffer.  Circuits of up to 1024 qubits.
 *
 * sp_symbolize_device_work_bytes: the work-buffer size that always holds the
 * tableau, the phase rows (n_qubits x ceil((n_vars + 1)/64) uint64 words at
 * most) and the outcome records, plus room for the index lists of
 * determined outcomes (their worst case, capped at 2^26 entries).
 *
 * sp_symbolize_device: d_work is device memory, 256-byte aligned, of
 * work_bytes bytes (any size at least the fixed part; what is left holds the
 * index lists); the library clears and uses it, and it is free again when
 * the call returns.  The call is synchronous with respect to the host: it
 * uploads the instruction stream, runs the kernel, copies the results back
 * and assembles the model on the host (column lists, output rows) like
 * sp_symbolize_outputs.  *out is owned by the caller (sp_model_free).
 * Errors: SP_E_INVALID (null, misaligned or too small buffer, unknown
 * outputs), SP_E_LIMIT (more than 1024 qubits or 2^24 variables, or the
 * lists outgrow the buffer: the message gives a size that suffices),
 * SP_E_NOMEM, SP_E_DEVICE. */
int sp_symbolize_device_work_bytes(const sp_circuit* circuit, size_t* bytes);
int sp_symbolize_device(const sp_circuit* circuit, int outputs, void* d_work, size_t work_bytes, void* stream,
                        sp_model** out);

/* How sp_symbolize_device runs (same model either way):
 *   SP_INIT_ONE_PASS  one workgroup updates tableau and phase rows together;
 *   SP_INIT_TWO_PASS  the one-workgroup pass only logs each row operation's
 *                     rows (the tableau never depends on the phases, Fact 2),
 *                     then a kernel over the whole GPU replays the log on the
 *                     phase rows, each workgroup a slice of their words in
 *                     LDS, and two small kernels turn the determined
 *                     outcomes' rows into index lists;
 *   SP_INIT_AUTO      two passes when the phase rows (n_qubits x
 *                     ceil((variables + 1)/64) words) exceed 64 KiB.
 * The two-pass work buffer holds the log (with the fault snapshots and, per
 * 64 variables, where the log introduces them, so that each replay slice
 * starts there) and, after it, the determined recorded outcomes' rows and
 * lists; sp_symbolize_device_work_bytes_mode
 * sizes that room for every recorded outcome, at most 1 GiB; a call that
 * needs more fails with SP_E_LIMIT.
 *
 * need_bytes (nullable, host): set on every return.  When the call fails
 * because work_bytes is too small -- SP_E_INVALID for the fixed part,
 * SP_E_LIMIT for the rows and lists of determined outcomes -- it holds a
 * work-buffer size that suffices for the failed step (a second call with
 * that size may still name a larger one once the lists' length is known);
 * otherwise 0. */
enum { SP_INIT_AUTO = 0, SP_INIT_ONE_PASS = 1, SP_INIT_TWO_PASS = 2 };
int sp_symbolize_device_work_bytes_mode(const sp_circuit* circuit, int mode, size_t* bytes);
int sp_symbolize_device_mode(const sp_circuit* circuit, int outputs, int mode, void* d_work, size_t work_bytes,
                             void* stream, sp_model** out, size_t* need_bytes);

int sp_model_dims(const sp_model* model, sp_dims* out);

/* Expected work of one 64-shot word: fired locations (sum over drawn
 * locations of 1 - (1 - q)^64, q = T_m / 2^32) and the (row, variable)
 * entries they touch on the sparse path.  Used to size and key launch
 * tuning; exact arithmetic is not needed here. */
int sp_model_expected_work(const sp_model* model, double* fired_per_word, double* entries_per_word);

/* Dense export of M and c: M has n_meas rows of row_words uint64 words
 * (row_words >= ceil(n_vars/64)); bit j of row k is M[k][j].  c (nullable):
 * ceil(n_meas/64) words, bit k = constant term of measurement k.  Host memory. */
int sp_model_export_dense(const sp_model* model, uint64_t* M, size_t row_words, uint64_t* c);

/* Column-list (CSC) export: col_ptr has n_vars+1 entries, row_idx nnz entries
 * (ascending rows within a column).  Host memory. */
int sp_model_export_csc(const sp_model* model, uint32_t* col_ptr, uint32_t* row_idx);

/* Variable j belongs to location var_loc[j], code bit var_bit[j].  Host memory. */
int sp_model_export_vars(const sp_model* model, uint32_t* var_loc, uint8_t* var_bit);

/* Bytes of device memory the resident model needs for `path`. */
int sp_model_device_bytes(const sp_model* model, int path, size_t* bytes);

/* Copies the model into the caller's device buffer d_buf (>= device_bytes,
 * 256-byte aligned) on `stream` and returns a handle that refers to it.  The
 * caller keeps d_buf alive and unmodified until sp_dmodel_free.  The copy is
 * asynchronous on `stream`; the host model may be freed after the call
 * returns (staging is internal and synchronous with respect to the host).
 *
 * Row tiles: the sampling kernel keeps a 64-shot word's output rows in one
 * LDS slab (17,920 rows at most on gfx950 with room for 16 waves' record
 * queues).  A model of more than 8,960 rows (two 8-wave workgroups' slabs
 * and queues per CU) is stored as row tiles of 3,840 rows (four per CU);
 * each tile holds only the locations
 * that reach its rows, and sp_sample samples every tile in one launch (the
 * buffer then also holds a table of the tiles' descriptors).  The draws are
 * keyed by location, so the output is the same bit for bit whatever the
 * tiling.
 * Errors: SP_E_INVALID, SP_E_LIMIT (a tile does not fit the device's LDS,
 * more than 2^27 rows), SP_E_DEVICE. */
int sp_model_upload(const sp_model* model, int path, void* d_buf, size_t buf_bytes, void* stream,
                    sp_dmodel** out);
/* The same with an explicit tile size: tile_rows = 0 chooses as above,
 * otherwise tiles of tile_rows rows (a multiple of 64, at most 19,456).
 * Errors as above, and SP_E_INVALID for another tile_rows. */
int sp_model_device_bytes_tiled(const sp_model* model, int path, uint32_t tile_rows, size_t* bytes);
int sp_model_upload_tiled(const sp_model* model, int path, uint32_t tile_rows, void* d_buf, size_t buf_bytes,
                          void* stream, sp_dmodel** out);
void sp_dmodel_free(sp_dmodel* dmodel);
int sp_dmodel_dims(const sp_dmodel* dmodel, sp_dims* out);
/* Row tiles of a device model and the rows of the largest (either pointer
 * may be NULL).  Errors: SP_E_INVALID. */
int sp_dmodel_tiles(const sp_dmodel* dmodel, uint32_t* n_tiles, uint32_t* rows_max);

/* Algorithm 1, Sampling, for shots [first_shot, first_shot + shots): draws
 * the variables of every drawn location from the keyed Philox stream, packs
 * them 64 shots per word and writes out = M s + c over GF(2) into d_out
 * (device, n_meas rows of ld_words words, 8-byte aligned,
 * ld_words >= ceil(shots/64)).  Asynchronous on `stream`.  The result is a
 * pure function of (model, seed, first_shot, shots).  shots = 0 is a no-op.
 * Each workgroup writes one word (or 2 or 4) of every row, so a row stride
 * of a large power of two (ld_words = 16,384 for 2^20 shots) sends the
 * lines written together to a few L2 sets, which write them back several
 * times; a stride of an odd number of 128-byte lines (ld_words = 16,400
 * there) writes each line once.
 * Errors: SP_E_INVALID, SP_E_LIMIT, SP_E_DEVICE. */
int sp_sample(const sp_dmodel* dmodel, uint64_t seed, uint64_t first_shot, uint64_t shots,
              uint64_t* d_out, size_t ld_words, void* stream);

/* Algorithm 1, Sampling, on the host CPU: the same draws, the same product
 * out = M s + c over GF(2) (Section 3.2.3, Eq. 4) and the same output as
 * sp_sample, computed from the host model's column lists by n_threads
 * threads (<= 0: one per hardware thread), 64 shots per word at a time (the
 * paper's own sampler is a sparse product on a CPU, Section 5).  h_out is
 * host memory of n_meas rows of ld_words uint64 words, laid out as for
 * sp_sample (ld_words >= ceil(shots/64); bits of shots >= `shots` written as
 * 0, words past the last one untouched).  Synchronous.  The result is a pure
 * function of (model, seed, first_shot, shots): bit for bit what sp_sample
 * writes for the same arguments.  shots = 0 is a no-op.  It is a separate
 * entry point, never a fallback: sp_sample does not call it.
 * Errors: SP_E_INVALID (null, ld_words too small, shot range past 2^64),
 * SP_E_LIMIT, SP_E_NOMEM. */
int sp_sample_host(const sp_model* model, uint64_t seed, uint64_t first_shot, uint64_t shots, uint64_t* h_out,
                   size_t ld_words, int n_threads);

/* Launch shape of the sampling kernel: a workgroup of waves_per_group
 * wave64s (1..16) owns words_per_group (1, 2 or 4) consecutive 64-shot words,
 * each with its own LDS slab of one row tile's uint64 rows (sparse path:
 * plus a 512-byte event queue per wave).  The output does not depend on the launch
 * shape. */
typedef struct {
  uint32_t waves_per_group;
  uint32_t words_per_group;
} sp_launch;

/* Read / set the launch shape used by sp_sample for this model (NULL resets
 * the library default).  Errors: SP_E_INVALID, SP_E_LIMIT (slabs exceed LDS). */
int sp_dmodel_get_launch(const sp_dmodel* dmodel, sp_launch* out);
int sp_dmodel_set_launch(sp_dmodel* dmodel, const sp_launch* launch);

/* ---- many circuits per launch (multi-circuit scheduling) ------------------ */

/* One sampling job: the same arguments as sp_sample. */
typedef struct {
  const sp_dmodel* model;
  uint64_t seed;
  uint64_t first_shot;
  uint64_t shots;
  uint64_t* d_out;
  size_t ld_words;
} sp_batch_item;

typedef struct sp_batch sp_batch;
typedef struct sp_graph sp_graph;

/* How a batched launch distributes word groups over workgroups. */
enum {
  SP_SCHED_PERSISTENT = 0, /* a device-filling grid; workgroups take tasks (runs of groups of one job)
                              from a device counter until none is left */
  SP_SCHED_FLAT = 1        /* one workgroup per group; the hardware dispatcher hands them out */
};

/* Device work memory (job table, task list or group-to-job map, counters)
 * for a batch of these items with the given launch shape (NULL = default)
 * and schedule.  Items with zero shots are dropped. */
int sp_batch_work_bytes(const sp_batch_item* items, size_t n, const sp_launch* launch, int schedule, size_t* bytes);

/* Builds a batch: every item's output is exactly what sp_sample would write
 * for it, and all items of one evaluation path are sampled by a single
 * launch (a batch mixing sparse- and dense-path models issues two).  Jobs
 * are ordered heaviest first.  d_work: caller's device buffer (>= work_bytes,
 * 256-byte aligned), written here on `stream` (synchronously with respect to
 * the host) and owned by the batch until sp_batch_free.  The models and
 * outputs must outlive the batch.  Errors: SP_E_INVALID, SP_E_LIMIT,
 * SP_E_DEVICE. */
int sp_batch_create(const sp_batch_item* items, size_t n, const sp_launch* launch, int schedule, void* d_work,
                    size_t work_bytes, void* stream, sp_batch** out);
/* Jobs kept, total word groups, persistent grid size, launch shape. */
int sp_batch_info(const sp_batch* batch, uint32_t* n_jobs, uint32_t* total_groups, uint32_t* grid, sp_launch* launch);
/* Queues the batched launch on `stream`.  The kernel resets its own work
 * counters, so a batch may be launched any number of times and replayed from
 * a captured graph; launches of one batch must not overlap in time. */
int sp_batch_launch(const sp_batch* batch, void* stream);
void sp_batch_free(sp_batch* batch);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the batched launch
 * of sp_batch_create + sp_batch_launch in one call, with the batch's job
 * table, task list or group map and work counters in a static device array
 * of the library (4 MiB on each GPU it runs on, held until the process
 * ends) instead of a caller's work buffer.  It allocates no device memory.
 * Items, launch shape (NULL = default) and schedule are as for
 * sp_batch_create, and every item's output is exactly what sp_sample writes
 * for it.  The tables are copied on `stream` and the call waits for that
 * copy (so also for earlier work on `stream`); the launch is then queued
 * asynchronously.  All calls on one GPU share the array: calls in order on
 * one stream are safe, calls on different streams or threads that overlap
 * in time race.  Errors: SP_E_INVALID, SP_E_LIMIT (the tables exceed
 * 4 MiB, or the slabs exceed the LDS), SP_E_NOMEM, SP_E_DEVICE. */
int sp_sample_batch_static(const sp_batch_item* items, size_t n, const sp_launch* launch, int schedule,
                           void* stream);

/* Captured launch sequences (HIP graphs).  capture_batch records one
 * sp_batch_launch; capture_plain records one sp_sample per item, in order.
 * Capture happens on a private stream; sp_graph_launch replays on `stream`. */
int sp_graph_capture_batch(const sp_batch* batch, sp_graph** out);
int sp_graph_capture_plain(const sp_batch_item* items, size_t n, sp_graph** out);
int sp_graph_launch(const sp_graph* graph, void* stream);
void sp_graph_free(sp_graph* graph);

/* ---- serving: resident models, HBM-budget admission, continuous batching --- */

typedef struct sp_server sp_server;

typedef struct {
  uint32_t max_active; /* requests sampled concurrently ("slots"), >= 1 */
  uint32_t max_queued; /* waiting requests before submit refuses (0 = 2^20) */
  uint64_t tick_cost;  /* work per launch tick in Philox block-words, i.e. the
                          model's blocks times 64-shot words (0 = 2^24) */
  sp_launch launch;    /* launch shape of the tick kernels ({0,0} = {8,1}) */
} sp_server_config;

enum { SP_REQ_QUEUED = 0, SP_REQ_ACTIVE = 1, SP_REQ_DONE = 2, SP_REQ_FAILED = 3 };

typedef struct {
  int state;              /* SP_REQ_* */
  uint32_t n_meas;
  uint64_t* d_out;        /* the request's output in the arena once admitted:
                             n_meas rows of ld_words words, layout of sp_sample
                             with first_shot as submitted; valid until release */
  uint64_t ld_words;      /* ceil(shots / 64) */
  uint64_t t_submit_ns;   /* host steady clock at submit */
  uint64_t t_admit_ns;    /* ... when the request got a slot and arena space */
  uint64_t t_done_ns;     /* ... when the scheduler saw its last words written */
} sp_request_status;

typedef struct {
  uint32_t queued, active;
  uint64_t arena_in_use, arena_capacity;
  uint64_t ticks, groups_launched, words_launched;
} sp_server_counters;

/* Device work memory the server needs for its per-tick job tables. */
int sp_server_work_bytes(const sp_server_config* cfg, size_t* bytes);

/* Starts a server on the current device.  d_arena (caller's device buffer,
 * 256-byte aligned) holds request outputs; a request is admitted, first in
 * first out, when a slot is free and its output (n_meas * ceil(shots/64) *
 * 8 bytes) fits.  A scheduler thread launches ticks on a private stream:
 * each tick samples a fair share of every active request's remaining words
 * with one batched launch per evaluation path, three ticks in flight on three streams.  Both
 * buffers are owned by the server until sp_server_destroy.  Models submitted
 * must stay alive until their requests are released.  Errors: SP_E_INVALID,
 * SP_E_NOMEM, SP_E_DEVICE. */
int sp_server_create(const sp_server_config* cfg, void* d_arena, size_t arena_bytes, void* d_work, size_t work_bytes,
                     sp_server** out);
/* Queues a request (thread-safe, does not block on the device).  Its output
 * is bit for bit what sp_sample(model, seed, first_shot, shots) writes.  A
 * row-tiled model is served whole: each word of its shot range costs one
 * workgroup per tile.  Errors: SP_E_INVALID, SP_E_LIMIT (slabs exceed the
 * LDS with the server's launch shape, or more row tiles than a tick's
 * 65,536 workgroups), SP_E_BUDGET (can never fit the arena, or the queue is
 * full). */
int sp_server_submit(sp_server* server, const sp_dmodel* model, uint64_t seed, uint64_t first_shot, uint64_t shots,
                     uint64_t* ticket);
int sp_server_status(sp_server* server, uint64_t ticket, sp_request_status* out);
/* Blocks until the request is done or failed (timeout_ms < 0: no limit).
 * Errors: SP_E_TIMEOUT, SP_E_DEVICE (the request failed), SP_E_INVALID. */
int sp_server_wait(sp_server* server, uint64_t ticket, int64_t timeout_ms, sp_request_status* out);
/* Frees a finished request's arena space; its output pointer is invalid
 * afterwards. */
int sp_server_release(sp_server* server, uint64_t ticket);
int sp_server_stats(sp_server* server, sp_server_counters* out);
/* Finishes the ticks in flight, fails requests that never ran, stops the
 * thread and frees the server's host resources. */
void sp_server_destroy(sp_server* server);

const char* sp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

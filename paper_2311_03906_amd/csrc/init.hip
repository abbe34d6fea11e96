// Initialization of Algorithm 1 on the GPU (Section 3.2.2: Init-C, Init-P,
// Init-M), producing the same model as the host pass.
//
// One workgroup of 1024 threads walks the circuit in program order; every
// branch depends only on the instruction stream, so all threads reach every
// barrier.  Layout, in a caller-provided device buffer:
//   X, Z  the tableau bit-packed down the rows, column-major: X[q] holds bit
//         r of qubit q's x-part for tableau rows r = 0..2n-1 (destabilizers
//         0..n-1, stabilizers n..2n-1) in RW = ceil(2n/64) words.  A gate on
//         qubit q is then a handful of word operations on column q, and the
//         row operations of a measurement are masked XORs on every column.
//   C     the constant phase bit of each row (RW words, kept in LDS).
//   P     the symbol part of each stabilizer's phase, one dense bit row of W
//         words per stabilizer (bit j = variable j): the (n_s+1)-bit phase
//         rows of Eq. 3 without the constant.
//   E     the expression of a determined measurement (two alternating
//         buffers of W words).
// Destabilizer phases are never read (as on the host).
//
// Init-P: the fault variable j on qubit q adds s_j to the stabilizer rows
// it anticommutes with.  A fault instruction's variables are consecutive, so
// each wave takes a 64-variable word of P: every lane gathers its variable's
// column word (z_q for X, x_q for Z) and a 64x64 bit transpose across the
// wave turns the block into the 64 rows' words.
//
// Init-M, random branch (a stabilizer row p has x_q = 1): the g sums of
// every row against p are accumulated at once as 2-bit bit-sliced counters
// over the rows, column by column; rows with x_q = 1 then take row p
// (x/z by masked XORs, the constant with the g correction, the symbols by
// XORing P rows); p's stabilizer becomes the destabilizer and p becomes Z_q
// with the fresh variable.  Determined branch: each column thread runs the
// ordered product of the stabilizers selected by the destabilizers' x_q bits
// for its own column, a reduction adds the g sums mod 4, and E is the XOR of
// the selected P rows; recorded outcomes are written as sorted index lists.
// Reset is measure then X^e; a Pauli controlled by record k is P^{e_k}.
//
// Two passes (large phase rows): the tableau never depends on the phases
// (Fact 2), so a logged pass runs the tableau alone and logs each row
// operation, and a replay kernel rebuilds the phase rows, each workgroup a
// slice of their words.  The logged pass takes runs of determined outcomes
// of one instruction together (the tableau does not change along them),
// one per wave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sp_internal.hpp"

namespace sp {
int set_error(int code, const std::string& msg);
}
using sp::set_error;
using sp::Op;
using sp::OpKind;

namespace {

constexpr uint32_t kThreads = 1024;
// Column words x selected rows up to which one wave computes a determined
// outcome of a run in the logged pass.
constexpr uint32_t kSoloWork = 64;
constexpr uint32_t kTargetChunk = 1024;   // measurement targets staged in LDS at a time
constexpr uint32_t kMaxQubits = 1024;
constexpr uint32_t kMaxRW = 2 * kMaxQubits / 64;   // 32
constexpr uint32_t kMaxDW = kMaxQubits / 64;       // words of a phase-row mask at most
constexpr uint32_t kChunks = 32;                   // kMaxRW x kChunks: the random branch's chunk counters
constexpr uint32_t kMaxChunks = 64;                // column chunks of the random-branch g sums, at most
constexpr size_t kStaticLds = 32 * 1024;           // at least the kernel's static LDS
constexpr uint32_t kPairStride = 34;               // a wave's column pairs: 64 columns and three pads, rounded up

// Device instruction stream: a header word (opcode | count << 8), then
// `count` items.
enum DevOp : uint32_t {
  D_H = 1, D_S, D_PX, D_PY, D_PZ,   // items: qubits (distinct within one instruction)
  D_CX,                             // items: a | b << 16 (no qubit twice within one instruction)
  D_FAULT,                          // items: q1 | q2 << 14 | kind << 28 (one location each)
  D_M, D_R, D_MR,                   // items: qubits (one location each, in order)
  D_FB                              // items: two words each, record index, then q | pauli << 16
};
enum FaultKind : uint32_t { F_X = 1, F_Y = 2, F_Z = 3, F_DEP1 = 4, F_DEP2 = 5 };

struct InitDev {
  const uint32_t* ops;
  uint32_t n_words;
  uint32_t n, RW, W;
  uint64_t* X;
  uint64_t* Z;
  uint64_t* P;
  uint64_t* E;
  int32_t* loc_var0;
  int32_t* rec_var;     // variable of a random recorded outcome, else -1
  uint32_t* rec_off;    // determined outcome: start of its list
  uint32_t* rec_len;
  uint32_t* rec_c;      // constant bit
  uint32_t* list;
  uint32_t list_cap;
  uint32_t* status;     // n_vars, n_random, list used, overflow, n_locs, n_rec, then (logged pass)
                        // log words and snapshot words (64-bit each, as two halves), recorded determined outcomes
  // Logged pass only (the phase rows are left to the replay kernel):
  uint64_t* log;        // row-operation log, see LogKind
  uint64_t* snap;       // per fault location and qubit: its x and z stabilizer-row masks
  uint64_t* first;      // per 64-variable word: 1 + the log position of the entry that introduces its first variable
  int32_t* rec_det;     // determined recorded outcome: its index among those, else -1
};

// Row-operation log of the logged pass.  Every mask is over the
// stabilizer rows, bit i = stabilizer row n + i = phase row i, in
// DW = ceil(n/64) words.  Entries, in program order:
//   FAULT   3 words: kind | fault kind << 8 | lg << 12 | nq << 16 | nv << 32;
//           first variable; snapshot offset (item k, qubit j: the x mask at
//           off + (k nq + j) 2 DW, the z mask after it)
//   RAND    2 words: kind | reset << 8 | (p - n) << 32; variable; then the
//           rows taking row p (x_a, without p), then (reset) the rows with z_a after
//   DET     2 words: kind | reset << 8 | recorded << 9 | det << 32; 0; then the
//           selected rows (destabilizers with x_a), then (reset) the rows with z_a
//   FB_RAND 2 words: kind | var << 32; 0; then the anticommuting rows
//   FB_DET  2 words: kind | det << 32; 0; then the anticommuting rows
//   RUN     1 word:  kind | r << 8: the next r (2..16) entries are DET entries
//           of one instruction computed together (along such a run the
//           tableau does not change)
enum LogKind : uint32_t { LOG_FAULT = 1, LOG_RAND, LOG_DET, LOG_FB_RAND, LOG_FB_DET, LOG_RUN };

__device__ __forceinline__ uint32_t bit_of(const uint64_t* col, uint32_t r) { return (uint32_t)(col[r >> 6] >> (r & 63)) & 1u; }

// Rows n..2n-1 of word w (the stabilizers).
__device__ __forceinline__ uint64_t stab_mask(uint32_t w, uint32_t n) {
  const uint32_t lo = w * 64, hi = lo + 64;
  uint64_t m = ~0ull;
  if (n > lo) m = (n >= hi) ? 0ull : (m << (n - lo));
  if (2 * n < hi) m &= (2 * n <= lo) ? 0ull : (~0ull >> (hi - 2 * n));
  return m;
}
// Rows 0..n-1 of word w (the destabilizers).
__device__ __forceinline__ uint64_t destab_mask(uint32_t w, uint32_t n) {
  const uint32_t lo = w * 64, hi = lo + 64;
  if (n <= lo) return 0ull;
  if (n >= hi) return ~0ull;
  return ~0ull >> (hi - n);
}

// g of the product (left) * (right) of one-qubit Paulis, as +1/-1 masks
// over rows: +1 for XY, YZ, ZX and -1 for XZ, YX, ZY (Aaronson-Gottesman).
__device__ __forceinline__ void g_masks(uint64_t lx, uint64_t lz, uint64_t rx, uint64_t rz, uint64_t& plus,
                                        uint64_t& minus) {
  plus = (lx & ~lz & rx & rz) | (lx & lz & ~rx & rz) | (~lx & lz & rx & ~rz);
  minus = (lx & ~lz & ~rx & rz) | (lx & lz & rx & ~rz) | (~lx & lz & rx & rz);
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return (uint64_t)uni((uint32_t)v) | (uint64_t)uni((uint32_t)(v >> 32)) << 32;
}
// Lane `src`'s value (src uniform).
__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t src) {
  return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)src) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)src) << 32;
}

// 64x64 bit transpose across a wave: lane l holds row l (bit j = column j)
// and gets back column l.  Six rounds; in the round of stride j, lanes l and
// l ^ j swap the blocks where the row index has bit j set and the column
// index has it clear (the recursive block transpose, LSB-first bits).
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, uint32_t j) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, (int)j, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), (int)j, 64);
  return (uint64_t)lo | (uint64_t)hi << 32;
}
__device__ __forceinline__ uint64_t transpose64(uint64_t x, uint32_t lane) {
  constexpr uint64_t kMask[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                                 0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const uint32_t j = 32u >> i;
    const uint64_t y = shfl_xor64(x, j);
    if (lane & j) x ^= ((y >> j) ^ x) & kMask[i];            // this lane holds the upper row of the pair
    else x ^= (((x >> j) ^ y) & kMask[i]) << j;               // the lower row
  }
  return x;
}

// A vector load of memory this kernel writes, also where the address is
// uniform (a scalar-cache load would not see the workgroup's own stores).
template <class T>
__device__ __forceinline__ T ld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Raw buffer access to one tableau half (n columns of RW words).  The
// hardware range check reads 0 for a byte offset at or beyond the buffer's
// size and drops such a store, so a lane with nothing to do is given an
// offset with bit 31 set instead of a branch.
constexpr uint32_t kBufWord3 = 0x00020000u;   // descriptor word 3: 32-bit data format, no swizzle
constexpr uint32_t kBeyond = 0x80000000u;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tab_rsrc(uint64_t* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, (int)kBufWord3);
}
__device__ __forceinline__ uint64_t buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
  return (uint64_t)v.x | (uint64_t)v.y << 32;
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t x) {
  u32x2 v;
  v.x = (uint32_t)x;
  v.y = (uint32_t)(x >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, 0);
}

// TAB_LDS: the tableau lives in dynamic LDS (2 n RW words), else in the
// work buffer.  LOG: the logged pass, which leaves the phase rows to the
// replay kernel and writes the row-operation log instead.
template <bool TAB_LDS, bool LOG>
__global__ void __launch_bounds__(kThreads) init_kernel(InitDev d) {
  extern __shared__ uint64_t s_tab[];
  __shared__ uint64_t s_C[kMaxRW];      // constant phase bit of every row
  __shared__ uint64_t s_mask[kMaxRW];   // x_a of every row but p, before a random measurement's update
  __shared__ uint64_t s_rpx[kMaxQubits / 64], s_rpz[kMaxQubits / 64];   // row p's x and z, bit q = column q
  __shared__ uint64_t s_c0[kMaxRW * kChunks];
  __shared__ uint64_t s_c1[kMaxRW * kChunks];
  __shared__ uint32_t s_rows[kMaxQubits];    // rows of the current measurement's row operations
  __shared__ uint32_t s_rows2[kMaxQubits];   // stabilizer rows with z_a, for a reset
  __shared__ uint32_t s_cnt[2];
  __shared__ uint32_t s_red[kThreads / 64];
  __shared__ uint32_t s_scan[kThreads / 64];
  __shared__ uint32_t s_tgt[kTargetChunk];   // targets of the current measurement instruction
  __shared__ uint32_t s_pair[kThreads / 64 * kPairStride];   // random outcome, tableau in global memory: each wave's column pairs
  const uint32_t tid = threadIdx.x;
  const uint32_t n = d.n, RW = d.RW, W = d.W;

  uint64_t* const X = TAB_LDS ? s_tab : d.X;
  uint64_t* const Z = TAB_LDS ? s_tab + (size_t)n * RW : d.Z;
  if (TAB_LDS) {
    for (uint32_t i = tid; i < 2 * n * RW; i += kThreads) s_tab[i] = 0;
    __syncthreads();
  }
  // |0...0>: destabilizer i = X_i, stabilizer i = Z_i (the work buffer arrives zeroed).
  if (tid < kMaxRW) s_C[tid] = 0;
  for (uint32_t q = tid; q < n; q += kThreads) {
    X[(size_t)q * RW + (q >> 6)] |= 1ull << (q & 63);
    Z[(size_t)q * RW + ((n + q) >> 6)] |= 1ull << ((n + q) & 63);
  }
  __syncthreads();

  uint32_t vars = 0, n_random = 0, nloc = 0, nrec = 0, listu = 0, overflow = 0;
  const uint32_t lane = tid & 63u, wave = tid >> 6;
  const uint32_t sw0 = n >> 6, sw1 = n ? (2 * n - 1) >> 6 : 0;   // words holding stabilizer rows
  // Logged pass: words of the log and of the snapshots written so far, and
  // determined recorded outcomes so far (all uniform).
  const uint32_t DW = (n + 63) >> 6, sh = n & 63u;
  uint64_t lp = 0, snp = 0;
  uint32_t n_det = 0;
  // Logged pass: a determined outcome that selects few rows is done by one
  // wave alone (the other waves walk past it), so a run of them costs no
  // barrier; a barrier rejoins the waves before the next step that reads
  // or writes shared state with every wave.
  bool solo_wrote = false;   // uniform
  auto join = [&]() {
    if (solo_wrote) __syncthreads();
    solo_wrote = false;
  };
  // Word k of a mask over phase-row indices (bit i = stabilizer row n + i),
  // from word(w) of the same mask over tableau rows.
  auto pword = [&](auto word, uint32_t k) -> uint64_t {
    const uint32_t w = sw0 + k;
    uint64_t v = word(w) >> sh;
    if (sh && w + 1 < RW) v |= word(w + 1) << (64u - sh);
    if (sh && k == DW - 1) v &= (1ull << sh) - 1ull;
    return v;
  };
  auto log_mask = [&](uint64_t at, auto word) {
    for (uint32_t k = tid; k < DW; k += kThreads) d.log[at + k] = pword(word, k);
  };

  // A uniform loop over the set stabilizer rows of a mask, run by every wave
  // alike (no barrier, no shared list): word(w) returns mask word w (a
  // uniform value).
  auto for_stab_rows = [&](auto word, auto body) {
    for (uint32_t w = sw0; n && w <= sw1; ++w) {
      uint64_t m = word(w) & stab_mask(w, n);
      while (m) {
        body(w * 64 + (uint32_t)__builtin_ctzll(m));
        m &= m - 1;
      }
    }
  };
  // Mask word w of the rows anticommuting with X^px Z^pz on qubit q.
  auto pauli_rows = [&](uint32_t q, uint32_t px, uint32_t pz, uint32_t w) -> uint64_t {
    return uni64((px ? ld(Z + (size_t)q * RW + w) : 0ull) ^ (pz ? ld(X + (size_t)q * RW + w) : 0ull));
  };

  // Wave 0 lists the set rows of a mask (its stabilizer or destabilizer
  // part) into dst, ascending, and the count into s_cnt[slot]; the others
  // read them after the next barrier.  word(w) returns mask word w, loaded
  // by lane w at once.
  auto rows_to_lds = [&](uint32_t* dst, uint32_t slot, auto word, bool stab) {
    if (wave == 0) {
      const uint64_t mw = lane < RW ? word(lane) & (stab ? stab_mask(lane, n) : destab_mask(lane, n)) : 0ull;
      uint32_t cnt = 0;
      for (uint32_t w = 0; w < RW; ++w) {
        const uint64_t m = readlane64(mw, w);
        if ((m >> lane) & 1u) dst[cnt + (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1))] = w * 64 + lane;
        cnt += (uint32_t)__builtin_popcountll(m);
      }
      if (lane == 0) s_cnt[slot] = cnt;
    }
  };
  // X^(px s) Z^(pz s) on qubit q for a single variable s adds s to the
  // stabilizer rows the Pauli anticommutes with (Fact 1).  Ends with a barrier.
  auto add_var = [&](uint32_t q, uint32_t px, uint32_t pz, uint32_t var) {
    if (tid < n) {
      const uint32_t row = n + tid;
      const uint32_t c = (px & bit_of(Z + (size_t)q * RW, row)) ^ (pz & bit_of(X + (size_t)q * RW, row));
      if (c) d.P[(size_t)tid * W + (var >> 6)] ^= 1ull << (var & 63);
    }
    __syncthreads();
  };

  for (uint32_t pc = 0; pc < d.n_words;) {
    const uint32_t hdr = uni(d.ops[pc]);
    const uint32_t op = hdr & 0xFFu, cnt = hdr >> 8;
    const uint32_t* it = d.ops + pc + 1;
    pc += 1 + cnt * (op == D_FB ? 2u : 1u);
    join();

    if (op == D_H || op == D_S || op == D_PX || op == D_PY || op == D_PZ || op == D_CX) {
      for (uint32_t i = tid; i < cnt * RW; i += kThreads) {
        const uint32_t k = i / RW, w = i % RW;
        const uint32_t item = it[k];
        if (op == D_CX) {
          const uint32_t a = item & 0xFFFFu, b = item >> 16;
          uint64_t& xa = X[(size_t)a * RW + w];
          uint64_t& za = Z[(size_t)a * RW + w];
          uint64_t& xb = X[(size_t)b * RW + w];
          uint64_t& zb = Z[(size_t)b * RW + w];
          const uint64_t vxa = xa, vza = za, vxb = xb, vzb = zb;
          const uint64_t t = vxa & vzb & ~(vxb ^ vza);
          if (t) atomicXor((unsigned long long*)&s_C[w], (unsigned long long)t);
          xb = vxb ^ vxa;
          za = vza ^ vzb;
        } else {
          uint64_t& x = X[(size_t)item * RW + w];
          uint64_t& z = Z[(size_t)item * RW + w];
          const uint64_t vx = x, vz = z;
          uint64_t t;
          if (op == D_H || op == D_S) t = vx & vz;
          else if (op == D_PX) t = vz;
          else if (op == D_PY) t = vx ^ vz;
          else t = vx;
          if (t) atomicXor((unsigned long long*)&s_C[w], (unsigned long long)t);
          if (op == D_H) {
            x = vz;
            z = vx;
          } else if (op == D_S) {
            z = vz ^ vx;
          }
        }
      }
      __syncthreads();
      continue;
    }

    if (op == D_FAULT) {
      // Every item of one instruction has the same channel kind, hence the
      // same number 2^lg of variables: item k owns vars + (k << lg) onward.
      const uint32_t kind0 = uni(it[0]) >> 28;
      const uint32_t lg = kind0 == F_DEP1 ? 1u : kind0 == F_DEP2 ? 2u : 0u;
      const uint32_t nv = cnt << lg;
      for (uint32_t k = tid; k < cnt; k += kThreads) d.loc_var0[nloc + k] = (int32_t)(vars + (k << lg));
      // One wave per 64-variable word of P.  Lane l takes variable
      // 64*vw + l and gathers the column word that decides which stabilizer
      // rows anticommute with its Pauli (z_q for X, x_q for Z, both for Y);
      // a 64x64 bit transpose turns those into row 64*w + j's bits for the
      // wave's 64 variables, held by lane j.
      if (LOG) {
        // Logged pass: the qubits' x and z stabilizer-row masks, for the
        // replay kernel to transpose into its own words of the phase rows.
        const uint32_t nq = kind0 == F_DEP2 ? 2u : 1u;
        const uint32_t per_item = nq * 2u * DW;
        for (uint32_t i = tid; i < cnt * per_item; i += kThreads) {
          const uint32_t k = i / per_item, rem = i % per_item;
          const uint32_t j = rem / (2u * DW), xz = (rem / DW) & 1u, w = rem % DW;
          const uint32_t item = it[k];
          const uint32_t q = j ? (item >> 14) & 0x3FFFu : item & 0x3FFFu;
          const uint64_t* col = (xz ? Z : X) + (size_t)q * RW;
          d.snap[snp + i] = pword([&](uint32_t ww) { return col[ww]; }, w);
        }
        if (tid == 0) {
          d.log[lp] = LOG_FAULT | kind0 << 8 | lg << 12 | nq << 16 | (uint64_t)nv << 32;
          d.log[lp + 1] = vars;
          d.log[lp + 2] = snp;
        }
        for (uint32_t w = (vars + 63) >> 6; nv && w <= (vars + nv - 1) >> 6; w += kThreads)
          if (w + tid <= (vars + nv - 1) >> 6) d.first[w + tid] = lp + 1;
        lp += 3;
        snp += (uint64_t)cnt * per_item;
        nloc += cnt;
        vars += nv;
        __syncthreads();
        continue;
      }
      const uint32_t lane = tid & 63u;
      const uint32_t vw0 = vars >> 6, vw1 = (vars + nv - 1) >> 6;
      const uint32_t sw0 = n >> 6, sw1 = (2 * n - 1) >> 6;
      for (uint32_t vw = vw0 + (tid >> 6); vw <= vw1; vw += kThreads / 64) {
        const uint32_t v = vw * 64 + lane;
        bool use_z = false, use_x = false;
        uint32_t qc = 0;
        if (v >= vars && v < vars + nv) {
          const uint32_t rel = v - vars, item = it[rel >> lg], b = rel & ((1u << lg) - 1u);
          const uint32_t kind = item >> 28;
          const uint32_t q = b >= 2 ? (item >> 14) & 0x3FFFu : item & 0x3FFFu;
          const bool xf = kind == F_X || kind == F_Y || ((kind == F_DEP1 || kind == F_DEP2) && !(b & 1u));
          const bool zf = kind == F_Z || kind == F_Y || ((kind == F_DEP1 || kind == F_DEP2) && (b & 1u));
          use_z = xf;
          use_x = zf;
          qc = q;
        }
        for (uint32_t w = sw0; w <= sw1; ++w) {
          uint64_t col = 0;
          if (use_z) col ^= Z[(size_t)qc * RW + w];
          if (use_x) col ^= X[(size_t)qc * RW + w];
          col &= stab_mask(w, n);
          if (__ballot(col != 0) == 0) continue;
          const uint64_t out = transpose64(col, lane);   // lane j: row 64 w + j's bits for the 64 variables
          const uint32_t row = w * 64 + lane;
          if (out) d.P[(size_t)(row - n) * W + vw] |= out;
        }
      }
      nloc += cnt;
      vars += nv;
      // The next instruction may rewrite the columns read above.
      __syncthreads();
      continue;
    }

    if (op == D_FB) {
      // Outcome records written by one thread are read by all below.
      __syncthreads();
      for (uint32_t k = 0; k < cnt; ++k) {
        const uint32_t rec = uni(it[2 * k]), qp = uni(it[2 * k + 1]);
        const uint32_t q = qp & 0xFFFFu, pauli = qp >> 16;   // 1 X, 2 Y, 3 Z
        const uint32_t px = pauli != 3, pz = pauli != 1;
        const int32_t rv = (int32_t)uni((uint32_t)ld(d.rec_var + rec));
        const uint32_t ec = uni(ld(d.rec_c + rec));
        if (LOG) {
          const uint32_t ref = rv >= 0 ? (uint32_t)rv : uni((uint32_t)ld(d.rec_det + rec));
          if (tid == 0) {
            d.log[lp] = (rv >= 0 ? LOG_FB_RAND : LOG_FB_DET) | (uint64_t)ref << 32;
            d.log[lp + 1] = 0;
          }
          log_mask(lp + 2, [&](uint32_t w) {
            return (px ? Z[(size_t)q * RW + w] : 0ull) ^ (pz ? X[(size_t)q * RW + w] : 0ull);
          });
          lp += 2 + DW;
          if (ec && tid < RW)
            s_C[tid] ^= ((px ? Z[(size_t)q * RW + tid] : 0ull) ^ (pz ? X[(size_t)q * RW + tid] : 0ull)) &
                        stab_mask(tid, n);
          __syncthreads();
          continue;
        }
        if (rv >= 0) {   // a random record: its variable alone, constant 0
          add_var(q, px, pz, (uint32_t)rv);
          continue;
        }
        // A determined record: its ascending index list, by words; the first
        // entry of each word gathers that word and adds it to the rows.
        const uint32_t off = uni(ld(d.rec_off + rec)), len = uni(ld(d.rec_len + rec));
        for (uint32_t i = tid; i < len; i += kThreads) {
          const uint32_t w = ld(d.list + off + i) >> 6;
          if (i == 0 || (ld(d.list + off + i - 1) >> 6) != w) {
            uint64_t e = 0;
            for (uint32_t j = i; j < len; ++j) {
              const uint32_t sj = ld(d.list + off + j);
              if ((sj >> 6) != w) break;
              e |= 1ull << (sj & 63);
            }
            for_stab_rows([&](uint32_t ww) { return pauli_rows(q, px, pz, ww); },
                          [&](uint32_t r) { d.P[(size_t)(r - n) * W + w] ^= e; });
          }
        }
        if (ec && tid < RW)
          s_C[tid] ^= ((px ? Z[(size_t)q * RW + tid] : 0ull) ^ (pz ? X[(size_t)q * RW + tid] : 0ull)) &
                      stab_mask(tid, n);
        __syncthreads();
      }
      continue;
    }

    // D_M, D_R, D_MR: one location per target, in order.  The targets are
    // staged in LDS, a chunk at a time, so that the serial chain of
    // measurements does not wait on a global load per target.
    for (uint32_t k = 0; k < cnt; ++k) {
      if (k % kTargetChunk == 0) {
        __syncthreads();   // every wave is done with the previous chunk
        solo_wrote = false;
        for (uint32_t i = tid; i < min(cnt - k, kTargetChunk); i += kThreads) s_tgt[i] = it[k + i];
        __syncthreads();
      }
      bool det0 = false;   // target k's outcome is determined (every wave checks, no barrier)
      if (LOG && TAB_LDS) {
        const uint32_t a0 = uni(s_tgt[k % kTargetChunk]);
        const uint64_t x0 = lane < RW ? ld(X + (size_t)a0 * RW + lane) & stab_mask(lane, n) : 0ull;
        det0 = __ballot(x0 != 0) == 0;
      }
      if (LOG && TAB_LDS && det0) {
        // A run of determined outcomes that select few rows, one per wave:
        // the tableau does not change along such a run, so every outcome's
        // g sums are computed at once; only C changes (a reset with outcome
        // 1 flips the rows with z_a), and wave 0 follows that chain in order
        // in registers.
        const uint32_t nb_max = min(min(cnt - k, kThreads / 64), kTargetChunk - k % kTargetChunk);
        const bool recorded = op != D_R, reset = op != D_M;
        uint64_t* const s_bsel = s_c0;         // [kMaxDW][kMaxDW]: selected rows (phase-row indices)
        uint64_t* const s_bzp = s_c0 + 256;    // [kMaxDW][kMaxDW]: rows with z_a (phase-row indices)
        join();   // the previous run's buffers are free
        uint64_t dm = 0;
        uint32_t aj = 0;
        if (wave < nb_max) {
          aj = uni(s_tgt[(k + wave) % kTargetChunk]);
          const uint64_t xw = lane < RW ? ld(X + (size_t)aj * RW + lane) : 0ull;
          const bool random = __ballot((lane < RW ? xw & stab_mask(lane, n) : 0ull) != 0) != 0;
          dm = lane < DW ? xw & destab_mask(lane, n) : 0ull;
          uint32_t ns = 0;
          for (uint32_t kk = 0; kk < DW; ++kk) ns += (uint32_t)__builtin_popcountll(readlane64(dm, kk));
          if (lane == 0) s_red[wave] = (!random && ns * DW <= kSoloWork) ? 1u : 0u;
        }
        __syncthreads();
        uint32_t r = 0;
        while (r < nb_max && s_red[r]) ++r;
        r = uni(r);
        if (r > 0) {
          if (wave < r) {
            // The product's g sums, bit-sliced: bit j of a lane's masks is
            // column lane + 64 j.
            uint32_t xs = 0, zs = 0, gs = 0;
            uint64_t words = __ballot(dm != 0);
            while (words) {
              const uint32_t kk = (uint32_t)__builtin_ctzll(words);
              words &= words - 1;
              uint64_t x = readlane64(dm, kk);
              while (x) {
                const uint32_t row = n + kk * 64 + (uint32_t)__builtin_ctzll(x);
                x &= x - 1;
                const uint32_t rw = row >> 6, rb = row & 63u;
                uint32_t xi = 0, zi = 0;
                constexpr uint32_t kCols = 4;   // columns' loads in flight
                for (uint32_t j = 0; j < DW; j += kCols) {
                  uint64_t xv[kCols], zv[kCols];
#pragma unroll
                  for (uint32_t u = 0; u < kCols; ++u) {
                    const uint32_t q = lane + 64 * (j + u);
                    const bool ok = j + u < DW && q < n;
                    xv[u] = ok ? X[(size_t)q * RW + rw] : 0ull;
                    zv[u] = ok ? Z[(size_t)q * RW + rw] : 0ull;
                  }
#pragma unroll
                  for (uint32_t u = 0; u < kCols; ++u) {
                    xi |= (uint32_t)((xv[u] >> rb) & 1u) << (j + u);
                    zi |= (uint32_t)((zv[u] >> rb) & 1u) << (j + u);
                  }
                }
                uint64_t plus, minus;
                g_masks(xi, zi, xs, zs, plus, minus);
                gs += (uint32_t)__builtin_popcountll(plus) - (uint32_t)__builtin_popcountll(minus);
                xs ^= xi;
                zs ^= zi;
              }
            }
            // The sum over lanes mod 4 (0 or 2), from the low bits' ballots.
            const uint32_t gsum = (uint32_t)__builtin_popcountll(__ballot(gs & 1u)) +
                                  2u * (uint32_t)__builtin_popcountll(__ballot(gs & 2u));
            if (lane == 0) s_red[wave] = 1u | ((gsum & 3u) == 2u ? 2u : 0u);
            if (lane < DW) {
              s_bsel[wave * kMaxDW + lane] = dm;
              if (reset) s_bzp[wave * kMaxDW + lane] = pword([&](uint32_t w) { return Z[(size_t)aj * RW + w]; }, lane);
            }
          }
          __syncthreads();
          if (wave == 0) {
            // C over phase-row indices (bit i: row n + i), lane kk word kk.
            uint64_t cp = lane < DW ? pword([&](uint32_t w) { return s_C[w]; }, lane) : 0ull;
            uint64_t ecm = 0;   // outcomes with constant 1
            for (uint32_t j = 0; j < r; ++j) {
              const uint64_t sel = lane < DW ? s_bsel[j * kMaxDW + lane] : 0ull;
              const uint32_t par = (uint32_t)__builtin_popcountll(__ballot(__builtin_popcountll(sel & cp) & 1u)) & 1u;
              if (par ^ ((s_red[j] >> 1) & 1u)) {
                ecm |= 1ull << j;
                if (reset && lane < DW) cp ^= s_bzp[j * kMaxDW + lane];
              }
            }
            // A run of two or more entries is announced by a RUN entry.
            const uint32_t ew = 2u + (reset ? 2u : 1u) * DW;   // log words per outcome
            const uint64_t lb = lp + (r > 1 ? 1u : 0u);
            if (r > 1 && lane == 0) d.log[lp] = LOG_RUN | r << 8;
            for (uint32_t i = lane; i < r * DW; i += 64) {
              const uint32_t j = i / DW, kk = i % DW;
              d.log[lb + j * ew + 2 + kk] = s_bsel[j * kMaxDW + kk];
              if (reset) d.log[lb + j * ew + 2 + DW + kk] = s_bzp[j * kMaxDW + kk];
            }
            if (lane < r) {
              const uint32_t j = lane;
              d.loc_var0[nloc + j] = -1;
              d.log[lb + j * ew] = LOG_DET | (reset ? 1u : 0u) << 8 | (recorded ? 1u : 0u) << 9 |
                                   (uint64_t)(recorded ? n_det + j : 0u) << 32;
              d.log[lb + j * ew + 1] = 0;
              if (recorded) {
                d.rec_var[nrec + j] = -1;
                d.rec_c[nrec + j] = (uint32_t)(ecm >> j) & 1u;
                d.rec_off[nrec + j] = 0;
                d.rec_len[nrec + j] = 0;
                d.rec_det[nrec + j] = (int32_t)(n_det + j);
              }
            }
            // Resets with outcome 1: X on qubit a flips C of the rows with z_a.
            if (reset && lane < RW) {
              uint64_t acc = 0;
              for (uint64_t em = uni64(ecm); em; em &= em - 1) {
                const uint32_t at = uni(s_tgt[(k + (uint32_t)__builtin_ctzll(em)) % kTargetChunk]);
                acc ^= Z[(size_t)at * RW + lane];
              }
              s_C[lane] ^= acc & stab_mask(lane, n);
            }
          }
          lp += (r > 1 ? 1u : 0u) + (uint64_t)r * (2u + (reset ? 2u : 1u) * DW);
          if (recorded) {
            n_det += r;
            nrec += r;
          }
          nloc += r;
          k += r - 1;
          solo_wrote = true;
          continue;
        }
      }
      const uint32_t a = uni(s_tgt[k % kTargetChunk]);
      const uint64_t* xa = X + (size_t)a * RW;
      // Pivot: the first stabilizer row with x_a = 1, found by every wave.
      uint32_t p = 0xFFFFFFFFu;
      {
        const uint64_t m = lane < RW ? ld(xa + lane) & stab_mask(lane, n) : 0ull;
        const uint64_t nz = __ballot(m != 0);
        if (nz) {
          const uint32_t w = (uint32_t)__builtin_ctzll(nz);
          p = w * 64 + (uint32_t)__builtin_ctzll(readlane64(m, w));
        }
        p = uni(p);
      }
      join();
      int32_t e_var = -1;
      uint32_t e_c = 0;
      const uint32_t Wt = (vars + 1 + 63) >> 6;   // words holding every variable so far, and one more
      // Two alternating buffers: a buffer is rewritten two measurements
      // later, after barriers every thread passes only once done with it.
      uint64_t* const Ecur = d.E + (size_t)(nloc & 1u) * W;

      if (p != 0xFFFFFFFFu) {
        // ---- random outcome: a fresh variable ------------------------------
        e_var = (int32_t)vars;
        if (tid == 0) d.loc_var0[nloc] = (int32_t)vars;
        ++vars;
        ++n_random;
        const uint32_t pw = p >> 6;
        const uint64_t pb = 1ull << (p & 63);
        if (!LOG) rows_to_lds(s_rows, 0, [&](uint32_t w) { return ld(xa + w) & ~(w == pw ? pb : 0ull); }, true);
        if (tid < RW) s_mask[tid] = ld(xa + tid) & ~(tid == pw ? pb : 0ull);
        const uint32_t cp = bit_of(s_C, p);
        // Row p's symbols move to Ecur, to be added to the rows below; row p
        // becomes the fresh variable alone.
        if (!LOG) {
          uint64_t* pp = d.P + (size_t)(p - n) * W;
          for (uint32_t w = tid; w < Wt; w += kThreads) {
            Ecur[w] = pp[w];
            pp[w] = w == ((uint32_t)e_var >> 6) ? 1ull << ((uint32_t)e_var & 63) : 0ull;
          }
        }
        // Row p's x and z in every column, one thread per column: only the
        // columns where row p has x or z add to the g sums below.
        uint64_t bxq = 0, bzq = 0, mx, mz;
        if (tid < n) {
          bxq = X[(size_t)tid * RW + pw] & pb;
          bzq = Z[(size_t)tid * RW + pw] & pb;
        }
        mx = __ballot(bxq != 0);
        mz = __ballot(bzq != 0);
        if (lane == 0) {
          s_rpx[wave] = mx;
          s_rpz[wave] = mz;
        }
        // Tableau in global memory: each wave lists its own 64 columns where
        // row p has x or z in pairs by row p's Pauli there (X, then Z, then
        // Y, each padded to an even count with an entry that names no
        // column); the wave then updates exactly those columns below.
        const uint32_t kxn = (uint32_t)__builtin_popcountll(mx & ~mz), kzn = (uint32_t)__builtin_popcountll(mz & ~mx),
                       kyn = (uint32_t)__builtin_popcountll(mx & mz);
        const uint32_t o1 = (kxn + 1) & ~1u, o2 = o1 + ((kzn + 1) & ~1u), npair = (o2 + ((kyn + 1) & ~1u)) / 2;
        if (!TAB_LDS) {
          uint16_t* const col = reinterpret_cast<uint16_t*>(s_pair + wave * kPairStride);
          const uint64_t below = (1ull << lane) - 1ull;
          if (bxq | bzq) {
            const uint32_t at = bzq == 0   ? (uint32_t)__builtin_popcountll(mx & ~mz & below)
                                : bxq == 0 ? o1 + (uint32_t)__builtin_popcountll(mz & ~mx & below)
                                           : o2 + (uint32_t)__builtin_popcountll(mx & mz & below);
            col[at] = (uint16_t)tid;
          }
          if (lane == 0) {
            if (kxn & 1u) col[kxn] = 0xFFFFu;
            if (kzn & 1u) col[o1 + kzn] = 0xFFFFu;
            if (kyn & 1u) col[o2 + kyn] = 0xFFFFu;
          }
        }
        __syncthreads();
        // g sums of every row against row p, bit-sliced mod 4, per (word, column
        // chunk), then added over the chunks.
        // Tableau in LDS: thread tid takes word tid % RW of chunk tid / RW, so
        // a wave's loads cover consecutive words and every lane works.
        // Tableau in global memory: a chunk is a wave (lane = word, both
        // halves added).
        const uint32_t nch = TAB_LDS ? min(kMaxChunks, kThreads / RW) : kThreads / 64;   // column chunks
        if (!TAB_LDS) {
          // In the columns where row p has x or z, one pass reads each word
          // once, adds it to the g sums and writes it updated: rows with x_a
          // take row p's x/z, destabilizer p-n becomes row p, row p becomes
          // Z_a.  A wave takes its own listed columns a pair at a time, one
          // column per half-wave: the g terms and the update then have one
          // form per pair and no branch, and a half-wave's loads and stores
          // cover a column's words (lane w: word w).  No other wave reads or
          // writes these columns before the next barrier.  In the other
          // columns only destabilizer p-n changes (it becomes row p's zeros).
          const uint32_t dr = p - n, dw = dr >> 6;
          const uint64_t db = 1ull << (dr & 63);
          if (tid < n && !(bxq | bzq)) {
            const uint64_t vx = X[(size_t)tid * RW + dw], vz = Z[(size_t)tid * RW + dw];
            if (vx & db) X[(size_t)tid * RW + dw] = vx & ~db;
            if (vz & db) Z[(size_t)tid * RW + dw] = vz & ~db;
          }
          const uint32_t w = lane & 31u, half = lane >> 5;
          const uint64_t mw = w < RW ? s_mask[w] : 0ull;   // x_a of every row but p
          const uint64_t dbm = w == dw ? db : 0ull, pbm = w == pw ? pb : 0ull;
          const uint64_t keep = ~(dbm | pbm), m1 = mw & keep;   // m1: rows taking row p, but the rewritten two
          // Byte offset of word w in a column, beyond the buffer where the
          // column's word cannot change; `fix` (or-ed into the store offset of
          // the half that changes only at the rewritten rows) likewise.
          const uint32_t live = (w < RW && (mw | dbm | pbm)) ? w * 8u : kBeyond;
          const uint32_t fix = (dbm | pbm) ? 0u : kBeyond;
          const uint32_t cb = RW * 8u;   // bytes per column
          const __amdgpu_buffer_rsrc_t rx = tab_rsrc(X, n * cb), rz = tab_rsrc(Z, n * cb);
          uint64_t c0 = 0, c1 = 0;
          // c += plus; c -= minus (mod 4, per bit)
          auto add = [&](uint64_t plus, uint64_t minus) {
            c1 ^= c0 & plus;
            c0 ^= plus;
            c1 ^= ~c0 & minus;
            c0 ^= minus;
          };
          // Pairs' loads in flight (fewer where the one-pass kernel keeps more
          // registers live for the phase rows).
          constexpr uint32_t kF = LOG ? 4 : 2;
          const uint32_t* const pairs = s_pair + wave * kPairStride;
          for (uint32_t s0 = 0; s0 < npair; s0 += kF) {
            uint32_t off[kF];
            uint64_t vx[kF], vz[kF];
            uint32_t isa = 0;   // bit i: pair i's column in this half is column a
#pragma unroll
            for (uint32_t i = 0; i < kF; ++i) {
              const uint32_t s = s0 + i;
              const uint32_t q = s < npair ? (pairs[s] >> (16u * half)) & 0xFFFFu : 0xFFFFu;
              off[i] = q * cb + live;   // beyond the tableau for a pad (q * cb >= n cb) or a dead lane
              isa |= (q == a ? 1u : 0u) << i;
              vx[i] = buf_ld(rx, off[i]);
              vz[i] = buf_ld(rz, off[i]);
            }
#pragma unroll
            for (uint32_t i = 0; i < kF; ++i) {
              const uint32_t s = s0 + i;
              if (s >= npair) break;
              const uint64_t x = vx[i], z = vz[i];
              const uint64_t pa = ((isa >> i) & 1u) ? pbm : 0ull;   // row p becomes Z_a
              if (2 * s < o1) {   // row p has X: +1 on Y, -1 on Z
                add(x & z, ~x & z);
                buf_st(rx, off[i], ((x ^ m1) & keep) | dbm);
                buf_st(rz, off[i] | fix, (z & keep) | pa);
              } else if (2 * s < o2) {   // Z: +1 on X, -1 on Y
                add(x & ~z, x & z);
                buf_st(rx, off[i] | fix, x & keep);
                buf_st(rz, off[i], ((z ^ m1) & keep) | dbm);
              } else {   // Y: +1 on Z, -1 on X
                add(~x & z, x & ~z);
                buf_st(rx, off[i], ((x ^ m1) & keep) | dbm);
                buf_st(rz, off[i], ((z ^ m1) & keep) | dbm | pa);
              }
            }
          }
          {   // the other half-wave's columns
            const uint64_t b0 = shfl_xor64(c0, 32), b1 = shfl_xor64(c1, 32);
            c1 ^= b1 ^ (c0 & b0);
            c0 ^= b0;
          }
          if (half == 0 && w < RW) {
            s_c0[w * nch + wave] = c0;
            s_c1[w * nch + wave] = c1;
          }
        } else {
          const uint32_t w = tid % RW, chunk = tid / RW;
          if (chunk < nch) {
            uint64_t c0 = 0, c1 = 0;
            const uint64_t mw = ld(xa + w) & ~(w == pw ? pb : 0ull);
            if (mw) {
              // c += plus; c -= minus (mod 4, per bit), for a column whose row-p
              // bits are (lx, lz) (all ones or zero) and whose word w is (vx, vz)
              auto add = [&](uint64_t lx, uint64_t lz, uint64_t vx, uint64_t vz) {
                uint64_t plus, minus;
                g_masks(lx, lz, vx, vz, plus, minus);
                c1 ^= c0 & plus;
                c0 ^= plus;
                c1 ^= ~c0 & minus;
                c0 ^= minus;
              };
              auto rp = [&](uint32_t q, uint64_t& lx, uint64_t& lz) {
                lx = ((s_rpx[q >> 6] >> (q & 63)) & 1u) ? ~0ull : 0ull;
                lz = ((s_rpz[q >> 6] >> (q & 63)) & 1u) ? ~0ull : 0ull;
              };
              uint32_t q = chunk;
              for (; q + nch < n; q += 2 * nch) {   // two columns' loads in flight
                uint64_t lx[2], lz[2], vx[2] = {0, 0}, vz[2] = {0, 0};
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                  const uint32_t qi = q + i * nch;
                  rp(qi, lx[i], lz[i]);
                  if (lx[i] | lz[i]) {
                    vx[i] = X[(size_t)qi * RW + w];
                    vz[i] = Z[(size_t)qi * RW + w];
                  }
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
                  if (lx[i] | lz[i]) add(lx[i], lz[i], vx[i], vz[i]);
              }
              for (; q < n; q += nch) {
                uint64_t lx, lz;
                rp(q, lx, lz);
                if (lx | lz) add(lx, lz, X[(size_t)q * RW + w], Z[(size_t)q * RW + w]);
              }
            }
            s_c0[w * nch + chunk] = c0;
            s_c1[w * nch + chunk] = c1;
          }
        }
        __syncthreads();
        // Constants of the rows taking row p (the sums are even for
        // commuting rows: bit 1 says "2 mod 4"); row p's becomes 0.  Four
        // threads per word each add a quarter of the chunk counters (2-bit
        // sums, bit-sliced), then two lane exchanges add the quarters.
        if (tid < 4 * kMaxRW) {
          const uint32_t w = tid / 4, qt = tid % 4;
          uint64_t c0 = 0, c1 = 0;
          if (w < RW) {
#pragma unroll 4
            for (uint32_t ch = qt; ch < nch; ch += 4) {
              const uint64_t b0 = s_c0[w * nch + ch], b1 = s_c1[w * nch + ch];
              c1 ^= b1 ^ (c0 & b0);
              c0 ^= b0;
            }
          }
          for (uint32_t off = 1; off < 4; off <<= 1) {
            const uint64_t b0 = shfl_xor64(c0, off), b1 = shfl_xor64(c1, off);
            c1 ^= b1 ^ (c0 & b0);
            c0 ^= b0;
          }
          if (qt == 0 && w < RW) {
            uint64_t cw = s_C[w] ^ (s_mask[w] & stab_mask(w, n) & (c1 ^ (cp ? ~0ull : 0ull)));
            if (w == pw) cw &= ~pb;
            s_C[w] = cw;
          }
        }
        // Symbols: every stabilizer row with x_a adds row p's old ones (the
        // logged pass logs those rows instead).
        if (LOG) {
          if (tid == 0) {
            d.log[lp] = LOG_RAND | (op != D_M ? 1u : 0u) << 8 | (uint64_t)(p - n) << 32;
            d.log[lp + 1] = (uint32_t)e_var;
            if ((e_var & 63) == 0) d.first[e_var >> 6] = lp + 1;
          }
          log_mask(lp + 2, [&](uint32_t w) { return s_mask[w]; });
        } else {
          const uint32_t nr = s_cnt[0];
          for (uint32_t i = tid; i < nr * Wt; i += kThreads) {
            const uint32_t r = s_rows[i / Wt], w = i % Wt;
            const uint64_t v = Ecur[w];
            if (v) d.P[(size_t)(r - n) * W + w] ^= v;
          }
        }
        // Tableau, one thread per column: rows with x_a take row p's x/z;
        // destabilizer p-n becomes row p; row p becomes Z_a (a tableau in
        // global memory was updated in the pass above).
        for (uint32_t q = tid; TAB_LDS && q < n; q += kThreads) {
          uint64_t* xq = X + (size_t)q * RW;
          uint64_t* zq = Z + (size_t)q * RW;
          const uint64_t bx = ((s_rpx[q >> 6] >> (q & 63)) & 1u) ? pb : 0ull;
          const uint64_t bz = ((s_rpz[q >> 6] >> (q & 63)) & 1u) ? pb : 0ull;
          const uint64_t lx = bx ? ~0ull : 0ull, lz = bz ? ~0ull : 0ull;
          if (bx | bz) {   // otherwise the column keeps its words
            for (uint32_t w = 0; w < RW; ++w) {
              const uint64_t m = s_mask[w];
              xq[w] ^= m & lx;
              zq[w] ^= m & lz;
            }
          }
          const uint32_t dr = p - n, dw = dr >> 6;
          const uint64_t db = 1ull << (dr & 63);
          xq[dw] = (xq[dw] & ~db) | (bx ? db : 0ull);
          zq[dw] = (zq[dw] & ~db) | (bz ? db : 0ull);
          xq[pw] &= ~pb;
          zq[pw] = (zq[pw] & ~pb) | (q == a ? pb : 0ull);
        }
        __syncthreads();
        if (op != D_R) {
          if (tid == 0) {
            d.rec_var[nrec] = e_var;
            d.rec_c[nrec] = 0;
            d.rec_off[nrec] = 0;
            d.rec_len[nrec] = 0;
            if (LOG) d.rec_det[nrec] = -1;
          }
          ++nrec;
        }
        // Reset (R, MR): X^e on qubit a, e the fresh variable.
        if (LOG) {
          if (op != D_M) {
            log_mask(lp + 2 + DW, [&](uint32_t w) { return Z[(size_t)a * RW + w]; });
            __syncthreads();
          }
          lp += 2 + (op != D_M ? 2u : 1u) * DW;
        } else if (op != D_M) {
          add_var(a, 1, 0, (uint32_t)e_var);
        }
      } else {
        // ---- determined outcome ----------------------------------------------
        // The product of the stabilizers n+i for the destabilizers i with
        // x_a = 1, in order: its g sums column by column (thread = column),
        // its constant, and its symbols E (each thread a range of words).
        if (tid == 0) d.loc_var0[nloc] = -1;
        rows_to_lds(s_rows, 0, [&](uint32_t w) { return ld(xa + w); }, false);
        if (LOG) {
          // The selected rows (destabilizers i with x_a: phase row i) and the
          // rows with z_a, logged while x_a and z_a cannot change.
          const bool recorded = op != D_R, reset = op != D_M;
          if (tid == 0) {
            d.log[lp] = LOG_DET | (reset ? 1u : 0u) << 8 | (recorded ? 1u : 0u) << 9 |
                        (uint64_t)(recorded ? n_det : 0u) << 32;
            d.log[lp + 1] = 0;
          }
          for (uint32_t k = tid; k < DW; k += kThreads) d.log[lp + 2 + k] = xa[k] & destab_mask(k, n);
          if (reset) log_mask(lp + 2 + DW, [&](uint32_t w) { return Z[(size_t)a * RW + w]; });
          lp += 2 + (reset ? 2u : 1u) * DW;
        } else if (op != D_M) {
          rows_to_lds(s_rows2, 1, [&](uint32_t w) { return ld(Z + (size_t)a * RW + w); }, true);
        }
        __syncthreads();
        const uint32_t ns = uni(s_cnt[0]);
        uint32_t g = 0, cpar = 0;
        if (tid < n) {
          const uint64_t* xq = X + (size_t)tid * RW;
          const uint64_t* zq = Z + (size_t)tid * RW;
          uint32_t xs = 0, zs = 0;
          auto step = [&](uint32_t xi, uint32_t zi) {
            uint64_t plus, minus;
            g_masks(xi, zi, xs, zs, plus, minus);
            g += (uint32_t)plus - (uint32_t)minus;   // mod 2^32, reduced mod 4 below
            xs ^= xi;
            zs ^= zi;
          };
          uint32_t j = 0;
          for (; j + 4 <= ns; j += 4) {   // four rows' loads in flight
            uint32_t xi[4], zi[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const uint32_t r = n + s_rows[j + i];
              xi[i] = bit_of(xq, r);
              zi[i] = bit_of(zq, r);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) step(xi[i], zi[i]);
          }
          for (; j < ns; ++j) step(bit_of(xq, n + s_rows[j]), bit_of(zq, n + s_rows[j]));
        }
        for (uint32_t j = 0; j < ns; ++j) cpar ^= bit_of(s_C, n + s_rows[j]);
        const uint32_t per = (Wt + kThreads - 1) / kThreads;
        const uint32_t w0 = min(Wt, tid * per), w1 = min(Wt, w0 + per);
        // This thread's words of E: the first two stay in registers, any
        // further ones (more than 2^17 variables) go to Ecur; only this
        // thread reads them back.
        uint64_t e0 = 0, e1 = 0;
        auto e_word = [&](uint32_t w) { return w == w0 ? e0 : w == w0 + 1 ? e1 : Ecur[w]; };
        uint32_t mine = 0;
        for (uint32_t w = w0; !LOG && w < w1; ++w) {
          uint64_t e = 0;
          uint32_t j = 0;
          for (; j + 4 <= ns; j += 4) {   // four independent loads in flight
            const uint64_t v0 = d.P[(size_t)s_rows[j] * W + w], v1 = d.P[(size_t)s_rows[j + 1] * W + w];
            const uint64_t v2 = d.P[(size_t)s_rows[j + 2] * W + w], v3 = d.P[(size_t)s_rows[j + 3] * W + w];
            e ^= v0 ^ v1 ^ v2 ^ v3;
          }
          for (; j < ns; ++j) e ^= d.P[(size_t)s_rows[j] * W + w];
          if (w == w0) e0 = e;
          else if (w == w0 + 1) e1 = e;
          else Ecur[w] = e;
          mine += (uint32_t)__builtin_popcountll(e);
        }
        const uint64_t g0 = __ballot(g & 1u), g1 = __ballot(g & 2u);
        if (lane == 0) s_red[wave] = (uint32_t)__builtin_popcountll(g0) + 2u * (uint32_t)__builtin_popcountll(g1);
        // Positions of the outcome's index list: a scan of the counts,
        // within each wave by shuffles, then over the waves' totals.
        uint32_t incl = mine;
        for (uint32_t off = 1; off < 64; off <<= 1) {
          const uint32_t y = __shfl_up(incl, off, 64);
          if (lane >= off) incl += y;
        }
        if (lane == 63) s_scan[wave] = incl;
        __syncthreads();
        uint32_t G = 0, before = 0, total = 0;
        for (uint32_t i = 0; i < kThreads / 64; ++i) {
          G += s_red[i];
          const uint32_t t = s_scan[i];
          before += i < wave ? t : 0u;
          total += t;
        }
        e_c = cpar ^ ((G & 3u) == 2u ? 1u : 0u);
        total = uni(total);
        if (LOG && op != D_R) {
          // The list comes from the replay kernel's rows of E.
          if (tid == 0) {
            d.rec_var[nrec] = -1;
            d.rec_c[nrec] = e_c;
            d.rec_off[nrec] = 0;
            d.rec_len[nrec] = 0;
            d.rec_det[nrec] = (int32_t)n_det;
          }
          ++n_det;
          ++nrec;
        } else if (op != D_R) {
          // The ascending list of E's set bits (each thread its own words).
          const bool fits = (uint64_t)listu + total <= d.list_cap;
          if (fits) {
            uint32_t pos = listu + before + incl - mine;
            for (uint32_t w = w0; w < w1; ++w) {
              uint64_t e = e_word(w);
              while (e) {
                d.list[pos++] = w * 64 + (uint32_t)__builtin_ctzll(e);
                e &= e - 1;
              }
            }
          } else {
            overflow = 1;
          }
          if (tid == 0) {
            d.rec_var[nrec] = -1;
            d.rec_c[nrec] = e_c;
            d.rec_off[nrec] = fits ? listu : 0u;
            d.rec_len[nrec] = fits ? total : 0u;
          }
          if (fits) listu += total;
          ++nrec;
        }
        // Reset (R, MR): X^e on qubit a adds e to the stabilizer rows with z_a.
        if (op != D_M) {
          const uint32_t nr = s_cnt[1];
          for (uint32_t w = w0; !LOG && w < w1; ++w) {
            const uint64_t e = e_word(w);
            if (!e) continue;
            uint32_t j = 0;
            for (; j + 4 <= nr; j += 4) {   // four independent read-modify-writes in flight
              uint64_t* p0 = d.P + (size_t)(s_rows2[j] - n) * W + w;
              uint64_t* p1 = d.P + (size_t)(s_rows2[j + 1] - n) * W + w;
              uint64_t* p2 = d.P + (size_t)(s_rows2[j + 2] - n) * W + w;
              uint64_t* p3 = d.P + (size_t)(s_rows2[j + 3] - n) * W + w;
              const uint64_t v0 = *p0, v1 = *p1, v2 = *p2, v3 = *p3;
              *p0 = v0 ^ e;
              *p1 = v1 ^ e;
              *p2 = v2 ^ e;
              *p3 = v3 ^ e;
            }
            for (; j < nr; ++j) d.P[(size_t)(s_rows2[j] - n) * W + w] ^= e;
          }
          if (e_c && tid < RW) s_C[tid] ^= Z[(size_t)a * RW + tid] & stab_mask(tid, n);
          __syncthreads();
        }
      }
      ++nloc;
    }
  }
  if (tid == 0) {
    d.status[0] = vars;
    d.status[1] = n_random;
    d.status[2] = listu;
    d.status[3] = overflow;
    d.status[4] = nloc;
    d.status[5] = nrec;
    d.status[6] = (uint32_t)lp;
    d.status[7] = (uint32_t)(lp >> 32);
    d.status[8] = (uint32_t)snp;
    d.status[9] = (uint32_t)(snp >> 32);
    d.status[10] = n_det;
  }
}

// ---- Replay of the log over the phase rows ---------------------------------
//
// The tableau never depends on the phases (Fact 2), so the logged pass can
// run ahead and the phase rows can be rebuilt afterwards from the log.  Each
// workgroup owns K consecutive 64-bit words of every phase row (P is n x W
// words; its slice, n x K words, lives in LDS) and applies the whole log to
// its slice; slices never interact.  A determined recorded outcome's words
// go to row `det` of E (n_det x W words) for the list kernels.
//
// The log is a chain of dependent steps, most of them small in a memory
// experiment (a determined outcome there selects two rows on average) and
// large in scrambling circuits (a random outcome's row list can hold half
// the rows).  A step touching at most kShortRows rows is done by wave 0
// alone: lane k owns word k of the slice, the rows come from scalar bit
// scans of the logged masks, and no barrier is needed.  Longer steps use
// every wave, with row lists in LDS and barriers.  All waves walk the log,
// so they take the same barriers; a barrier precedes any step after wave 0
// wrote alone.
struct ReplayArgs {
  const uint64_t* log;
  uint64_t log_words;
  const uint64_t* snap;
  const uint64_t* first;   // per variable word: 1 + the log position introducing its first variable
  uint64_t* E;             // [n_det][W], zero on entry
  uint32_t n, DW, K, W;
};

constexpr uint32_t kReplayThreads = 1024;
constexpr uint32_t kLogWindow = 1024;             // log words staged in LDS at a time
constexpr uint32_t kShortRows = 8;                // rows up to which one wave does a step
constexpr size_t kReplayStaticLds = 28 * 1024;   // at least the replay kernel's static LDS

__global__ void __launch_bounds__(kReplayThreads) replay_kernel(ReplayArgs r) {
  extern __shared__ uint64_t s_P[];   // [n][K]
  __shared__ uint32_t s_rows[kMaxQubits], s_rows2[kMaxQubits];
  __shared__ uint32_t s_cnt[2];
  __shared__ uint64_t s_part[kReplayThreads];
  __shared__ uint64_t s_E[64];
  __shared__ uint64_t s_log[kLogWindow];   // log words [win_lo, win_hi)
  __shared__ uint32_t s_rdm[kReplayThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t n = r.n, DW = r.DW, K = r.K;
  const uint32_t w_lo = blockIdx.x * K, Ks = min(K, r.W - w_lo);   // this slice: words [w_lo, w_lo + Ks)
  for (uint32_t i = tid; i < n * K; i += kReplayThreads) s_P[i] = 0;
  // Longest entry: a RUN of 16 entries of two header words and two masks.
  const uint64_t max_entry = 1u + 16u * (2u + 2u * DW);
  // Variables are numbered in the order the log introduces them, so before
  // the entry that introduces this slice's first variable every row is zero
  // in the slice and every entry leaves it so (its E words stay the zeros
  // E starts with): the walk starts there.
  const uint64_t f0 = r.first[w_lo];
  const uint64_t start = f0 ? min(f0 - 1, r.log_words) : 0;
  uint64_t win_lo = start, win_hi = start;
  bool solo_wrote = false;   // wave 0 wrote alone since the last barrier (uniform)
  // Every wave read row p of the slice to decide a skip since the last
  // barrier (uniform).  Any write to the slice must wait until all waves are
  // past that read: a wave that saw the row already changed would not skip,
  // and the waves would no longer meet the same barriers.
  bool read_pending = false;

  // Wave `wv` lists the set bits of a logged mask (DW words at m) into dst.
  auto list = [&](uint32_t wv, const uint64_t* m, uint32_t* dst, uint32_t slot) {
    if (wave == wv) {
      const uint64_t mw = lane < DW ? m[lane] : 0ull;
      uint32_t cnt = 0;
      for (uint32_t k = 0; k < DW; ++k) {
        const uint64_t x = readlane64(mw, k);
        if ((x >> lane) & 1u) dst[cnt + (uint32_t)__builtin_popcountll(x & ((1ull << lane) - 1))] = k * 64 + lane;
        cnt += (uint32_t)__builtin_popcountll(x);
      }
      if (lane == 0) s_cnt[slot] = cnt;
    }
  };
  // Set bits of a logged mask, counted by every wave (uniform).
  auto bits = [&](const uint64_t* m) {
    const uint64_t mw = lane < DW ? m[lane] : 0ull;
    uint32_t c = 0;
    for (uint32_t k = 0; k < DW; ++k) c += (uint32_t)__builtin_popcountll(readlane64(mw, k));
    return c;
  };
  // Wave 0 alone: f(i) for every set bit i of a logged mask, ascending (the
  // mask read once, lane k holding word k, and scanned with scalar ops).
  auto for_bits = [&](const uint64_t* m, auto f) {
    const uint64_t mw = lane < DW ? m[lane] : 0ull;
    uint64_t words = __ballot(mw != 0);
    while (words) {
      const uint32_t k = (uint32_t)__builtin_ctzll(words);
      words &= words - 1;
      uint64_t x = readlane64(mw, k);
      while (x) {
        f(k * 64 + (uint32_t)__builtin_ctzll(x));
        x &= x - 1;
      }
    }
  };
  // Row-parallel work: thread (rg, kw) takes word kw of the slice in rows
  // rg, rg + G, ... of a list (G row groups of K threads).
  const uint32_t G = kReplayThreads / K, rg = tid / K, kw = tid % K;
  const bool rk = rg < G && kw < Ks;
  // Rows dst[0..nr) of the slice ^= v(k).
  auto xor_rows = [&](const uint32_t* rows, uint32_t nr, auto v) {
    if (!rk) return;
    const uint64_t x = v(kw);
    uint32_t j = rg;
    for (; j + 3 * G < nr; j += 4 * G) {
      const uint32_t r0 = rows[j], r1 = rows[j + G], r2 = rows[j + 2 * G], r3 = rows[j + 3 * G];
      s_P[r0 * K + kw] ^= x;
      s_P[r1 * K + kw] ^= x;
      s_P[r2 * K + kw] ^= x;
      s_P[r3 * K + kw] ^= x;
    }
    for (; j < nr; j += G) s_P[rows[j] * K + kw] ^= x;
  };
  // Before a step that other waves take part in.
  auto join = [&]() {
    if (solo_wrote || read_pending) __syncthreads();
    solo_wrote = false;
    read_pending = false;
  };
  // Before wave 0 writes alone: every wave takes this barrier or none does,
  // since the skip that set read_pending was taken by all of them.
  auto settle = [&]() {
    if (read_pending) __syncthreads();
    read_pending = false;
  };
  const bool w0 = wave == 0, mine = w0 && lane < Ks;   // wave 0's lane = slice word
  __syncthreads();

  // The log is read through a window in LDS, refilled by all threads with
  // one coalesced load when the next entry may run past it (one load per
  // window instead of a dependent global load per entry).
  for (uint64_t lp = start; lp < r.log_words;) {
    if (lp + max_entry > win_hi && win_hi < r.log_words) {
      __syncthreads();   // every wave is done with the old window
      solo_wrote = false;
      read_pending = false;
      win_lo = lp;
      win_hi = min(lp + (uint64_t)kLogWindow, r.log_words);
      for (uint32_t i = tid; i < win_hi - win_lo; i += kReplayThreads) s_log[i] = r.log[win_lo + i];
      __syncthreads();
    }
    const uint64_t* e = s_log + (lp - win_lo);
    const uint64_t h0 = uni64(e[0]), h1 = uni64(e[1]);
    const uint32_t kind = (uint32_t)h0 & 0xFFu;
    const uint64_t* m = e + 2;
    if (kind == LOG_FAULT) {
      const uint32_t fk = ((uint32_t)h0 >> 8) & 0xFu, lg = ((uint32_t)h0 >> 12) & 0xFu, nq = ((uint32_t)h0 >> 16) & 0xFu;
      const uint32_t nv = (uint32_t)(h0 >> 32), v0 = (uint32_t)h1;
      const uint64_t off = uni64(e[2]);
      lp += 3;
      // One wave per variable word of the slice that the instruction covers;
      // lane l takes variable 64 vw + l, builds its anticommuting-row mask
      // from the snapshots, and the transpose gives each row's bits.
      const uint32_t vw0 = max(v0 >> 6, w_lo), vw1 = min((v0 + nv - 1) >> 6, w_lo + Ks - 1);
      if (nv == 0 || vw0 > vw1) continue;   // no variable of this slice
      join();
      for (uint32_t vw = vw0 + wave; vw <= vw1 && vw0 <= vw1; vw += kReplayThreads / 64) {
        const uint32_t v = vw * 64 + lane;
        bool xf = false, zf = false;
        const uint64_t* sx = r.snap;
        if (v >= v0 && v < v0 + nv) {
          const uint32_t rel = v - v0, item = rel >> lg, b = rel & ((1u << lg) - 1u);
          xf = fk == F_X || fk == F_Y || ((fk == F_DEP1 || fk == F_DEP2) && !(b & 1u));
          zf = fk == F_Z || fk == F_Y || ((fk == F_DEP1 || fk == F_DEP2) && (b & 1u));
          sx = r.snap + off + ((uint64_t)item * nq + (b >= 2 ? 1u : 0u)) * 2u * DW;
        }
        for (uint32_t k = 0; k < DW; ++k) {
          uint64_t col = 0;
          if (xf) col ^= sx[DW + k];   // an X fault flips the rows with z
          if (zf) col ^= sx[k];        // a Z fault the rows with x
          if (__ballot(col != 0) == 0) continue;
          const uint64_t out = transpose64(col, lane);
          const uint32_t row = k * 64 + lane;
          if (out && row < n) s_P[row * K + (vw - w_lo)] |= out;
        }
      }
      __syncthreads();
      continue;
    }
    if (kind == LOG_RUN) {
      // A run of DET entries of one instruction, one wave each: E of every
      // outcome from the rows before the run's resets; the resets then
      // follow in order on wave 0, where an outcome's E also takes the E of
      // every earlier reset whose rows with z_a meet its selected rows an
      // odd number of times.
      const uint32_t nr = ((uint32_t)h0 >> 8) & 0xFFu;
      const uint64_t lb = lp + 1;
      const bool reset = (h1 >> 8) & 1u;   // h1 is the first entry's header
      const uint32_t ew = 2u + (reset ? 2u : 1u) * DW;
      const uint64_t* e0 = s_log + (lb - win_lo);
      lp = lb + (uint64_t)nr * ew;
      join();
      uint64_t* const s_run = s_part;   // [16][64]: E of each outcome of the run
      if (wave < nr) {
        const uint64_t* ej = e0 + wave * ew;
        const uint64_t hj = uni64(ej[0]);
        uint64_t ev = 0;
        for_bits(ej + 2, [&](uint32_t i) {
          if (lane < Ks) ev ^= s_P[i * K + lane];
        });
        if (!reset) {
          if (((hj >> 9) & 1u) && lane < Ks) r.E[(size_t)(hj >> 32) * r.W + w_lo + lane] = ev;
        } else {
          s_run[wave * 64 + lane] = ev;
          const uint64_t sel = lane < DW ? ej[2 + lane] : 0ull;
          uint32_t dmask = 0;
          for (uint32_t j = 0; j < wave; ++j) {
            const uint64_t zj = lane < DW ? e0[j * ew + 2 + DW + lane] : 0ull;
            dmask |= ((uint32_t)__builtin_popcountll(__ballot(__builtin_popcountll(sel & zj) & 1u)) & 1u) << j;
          }
          if (lane == 0) s_rdm[wave] = dmask;
        }
      }
      __syncthreads();   // every wave is done reading the rows
      if (reset) {
        if (w0) {
          for (uint32_t j = 0; j < nr; ++j) {
            const uint64_t* ej = e0 + j * ew;
            const uint64_t hj = uni64(ej[0]);
            uint64_t ev = s_run[j * 64 + lane];
            const uint32_t dmask = uni(s_rdm[j]);
            if (dmask) {
              for (uint32_t dm = dmask; dm; dm &= dm - 1) ev ^= s_run[(uint32_t)__builtin_ctz(dm) * 64 + lane];
              s_run[j * 64 + lane] = ev;
            }
            if (((hj >> 9) & 1u) && lane < Ks) r.E[(size_t)(hj >> 32) * r.W + w_lo + lane] = ev;
            for_bits(ej + 2 + DW, [&](uint32_t i) {
              if (lane < Ks) s_P[i * K + lane] ^= ev;
            });
          }
        }
        solo_wrote = true;
      }
      continue;
    }
    const uint32_t flags = ((uint32_t)h0 >> 8) & 0xFFu, hi = (uint32_t)(h0 >> 32);
    if (kind == LOG_RAND) {
      const bool reset = flags & 1u;
      const uint32_t p = hi, var = (uint32_t)h1;
      lp += 2 + (reset ? 2u : 1u) * DW;
      const bool in = (var >> 6) >= w_lo && (var >> 6) < w_lo + Ks;
      const uint32_t vk = (var >> 6) - w_lo;
      const uint64_t vb = 1ull << (var & 63);
      // Row p zero in the slice and the variable elsewhere: nothing here
      // changes (most entries, for most slices).  Every wave reads the same
      // words, so all skip alike; the read needs no barrier unless wave 0
      // wrote alone since the last one, and the entry's own writes, if it is
      // not skipped, wait for every wave's read (read_pending).
      if (!in && !solo_wrote) {
        const uint64_t vp = lane < Ks ? s_P[p * K + lane] : 0ull;
        read_pending = true;
        if (__ballot(vp != 0) == 0) continue;
      }
      // The listed rows (row p is not among them) take row p's symbols; row p
      // becomes the fresh variable, which a reset then adds to the rows with
      // z_a instead.
      if (bits(m) + (reset ? bits(m + DW) : 0u) <= kShortRows) {
        settle();
        if (w0) {
          const uint64_t vp = mine ? s_P[p * K + lane] : 0ull;
          for_bits(m, [&](uint32_t i) {
            if (mine) s_P[i * K + lane] ^= vp;
          });
          if (mine) s_P[p * K + lane] = (!reset && in && lane == vk) ? vb : 0ull;
          if (reset && in)
            for_bits(m + DW, [&](uint32_t i) {
              if (i != p && lane == vk) s_P[i * K + vk] ^= vb;
            });
        }
        solo_wrote = true;
        continue;
      }
      join();
      {
        // Row p zero in the slice and the variable elsewhere: nothing here
        // changes (every wave reads the same words, so all skip alike).
        const uint64_t vp = lane < Ks ? s_P[p * K + lane] : 0ull;
        if (!in && __ballot(vp != 0) == 0) {
          read_pending = true;
          continue;
        }
      }
      list(0, m, s_rows, 0);
      if (reset) list(1, m + DW, s_rows2, 1);
      __syncthreads();
      xor_rows(s_rows, s_cnt[0], [&](uint32_t k) { return s_P[p * K + k]; });
      __syncthreads();
      for (uint32_t k = tid; k < Ks; k += kReplayThreads) s_P[p * K + k] = (!reset && in && k == vk) ? vb : 0ull;
      if (reset && in)
        for (uint32_t j = tid; j < s_cnt[1]; j += kReplayThreads)
          if (s_rows2[j] != p) s_P[s_rows2[j] * K + vk] ^= vb;
      __syncthreads();
      continue;
    }
    if (kind == LOG_DET) {
      const bool reset = flags & 1u, recorded = flags & 2u;
      lp += 2 + (reset ? 2u : 1u) * DW;
      // E = XOR of the selected rows; a reset adds it to the rows with z_a.
      if (bits(m) + (reset ? bits(m + DW) : 0u) <= kShortRows) {
        settle();
        if (w0) {
          uint64_t ev = 0;
          for_bits(m, [&](uint32_t i) {
            if (mine) ev ^= s_P[i * K + lane];
          });
          if (recorded && mine) r.E[(size_t)hi * r.W + w_lo + lane] = ev;
          if (reset)
            for_bits(m + DW, [&](uint32_t i) {
              if (mine) s_P[i * K + lane] ^= ev;
            });
        }
        solo_wrote = true;
        continue;
      }
      join();
      list(0, m, s_rows, 0);
      if (reset) list(1, m + DW, s_rows2, 1);
      __syncthreads();
      // Per (row group, word) partial sums, then per word (four independent
      // chains each, so the loads overlap).
      const uint32_t ns = s_cnt[0];
      if (rg < G) {
        uint64_t e0 = 0, e1 = 0, e2 = 0, e3 = 0;
        if (kw < Ks) {
          uint32_t j = rg;
          for (; j + 3 * G < ns; j += 4 * G) {
            const uint32_t r0 = s_rows[j], r1 = s_rows[j + G], r2 = s_rows[j + 2 * G], r3 = s_rows[j + 3 * G];
            e0 ^= s_P[r0 * K + kw];
            e1 ^= s_P[r1 * K + kw];
            e2 ^= s_P[r2 * K + kw];
            e3 ^= s_P[r3 * K + kw];
          }
          for (; j < ns; j += G) e0 ^= s_P[s_rows[j] * K + kw];
        }
        s_part[tid] = e0 ^ e1 ^ e2 ^ e3;
      }
      __syncthreads();
      if (tid < Ks) {
        uint64_t e0 = 0, e1 = 0, e2 = 0, e3 = 0;
        uint32_t gg = 0;
        for (; gg + 3 < G; gg += 4) {
          e0 ^= s_part[gg * K + tid];
          e1 ^= s_part[(gg + 1) * K + tid];
          e2 ^= s_part[(gg + 2) * K + tid];
          e3 ^= s_part[(gg + 3) * K + tid];
        }
        for (; gg < G; ++gg) e0 ^= s_part[gg * K + tid];
        const uint64_t ev = e0 ^ e1 ^ e2 ^ e3;
        s_E[tid] = ev;
        if (recorded) r.E[(size_t)hi * r.W + w_lo + tid] = ev;
      }
      __syncthreads();
      if (reset) {
        xor_rows(s_rows2, s_cnt[1], [&](uint32_t kk) { return s_E[kk]; });
        __syncthreads();
      }
      continue;
    }
    // LOG_FB_RAND / LOG_FB_DET: a Pauli conditioned on an earlier outcome.
    lp += 2 + DW;
    const bool in = (hi >> 6) >= w_lo && (hi >> 6) < w_lo + Ks;
    const uint32_t vk = (hi >> 6) - w_lo;
    const uint64_t vb = 1ull << (hi & 63);
    if (bits(m) <= kShortRows) {
      settle();
      if (w0) {
        if (kind == LOG_FB_DET) {
          const uint64_t ev = mine ? r.E[(size_t)hi * r.W + w_lo + lane] : 0ull;   // written by this lane
          for_bits(m, [&](uint32_t i) {
            if (mine) s_P[i * K + lane] ^= ev;
          });
        } else if (in) {
          for_bits(m, [&](uint32_t i) {
            if (lane == vk) s_P[i * K + vk] ^= vb;
          });
        }
      }
      solo_wrote = true;
      continue;
    }
    join();
    list(0, m, s_rows, 0);
    if (kind == LOG_FB_DET && tid < Ks) s_E[tid] = r.E[(size_t)hi * r.W + w_lo + tid];
    __syncthreads();
    if (kind == LOG_FB_DET) {
      xor_rows(s_rows, s_cnt[0], [&](uint32_t kk) { return s_E[kk]; });
    } else if (in) {
      for (uint32_t j = tid; j < s_cnt[0]; j += kReplayThreads) s_P[s_rows[j] * K + vk] ^= vb;
    }
    __syncthreads();
  }
}

// Index lists of the determined recorded outcomes from their rows of E:
// one workgroup per outcome counts its bits, the host scans the counts, and
// a second pass writes each row's set bits in ascending order.
constexpr uint32_t kListThreads = 256;

__global__ void __launch_bounds__(kListThreads) count_kernel(const uint64_t* E, uint32_t W, uint32_t* counts) {
  __shared__ uint32_t s_sum[kListThreads / 64];
  const uint64_t* row = E + (size_t)blockIdx.x * W;
  uint32_t c = 0;
  for (uint32_t w = threadIdx.x; w < W; w += kListThreads) c += (uint32_t)__builtin_popcountll(row[w]);
  for (uint32_t off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63u) == 0) s_sum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (uint32_t i = 0; i < kListThreads / 64; ++i) t += s_sum[i];
    counts[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kListThreads) write_lists_kernel(const uint64_t* E, uint32_t W, const uint32_t* offsets,
                                                                   uint32_t* list) {
  __shared__ uint32_t s_scan[kListThreads / 64];
  const uint64_t* row = E + (size_t)blockIdx.x * W;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t per = (W + kListThreads - 1) / kListThreads;
  const uint32_t w0 = min(W, tid * per), w1 = min(W, w0 + per);
  uint32_t mine = 0;
  for (uint32_t w = w0; w < w1; ++w) mine += (uint32_t)__builtin_popcountll(row[w]);
  uint32_t incl = mine;
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) s_scan[wave] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t i = 0; i < wave; ++i) before += s_scan[i];
  uint32_t pos = offsets[blockIdx.x] + before + incl - mine;
  for (uint32_t w = w0; w < w1; ++w) {
    uint64_t e = row[w];
    while (e) {
      list[pos++] = w * 64 + (uint32_t)__builtin_ctzll(e);
      e &= e - 1;
    }
  }
}

// The instruction stream for the kernel, with every instruction split into
// runs in which no qubit repeats (those run in parallel).
struct DevProgram {
  std::vector<uint32_t> words;
  uint64_t max_vars = 0;
  uint64_t list_bound = 0;   // most index entries the determined outcomes can need
  uint32_t n_rec = 0, n_locs = 0;
};

DevProgram compile(const sp_circuit& c) {
  DevProgram P;
  std::vector<uint32_t> seen(c.n_qubits + 1, 0);
  uint32_t stamp = 0;
  // One instruction per 2^20 items at most (the count has 24 bits).
  auto emit = [&](uint32_t op, const std::vector<uint32_t>& items, uint32_t per_item) {
    const size_t n_items = items.size() / per_item, step = 1u << 20;
    for (size_t i = 0; i < n_items; i += step) {
      const size_t k = std::min(step, n_items - i);
      P.words.push_back(op | (uint32_t)k << 8);
      P.words.insert(P.words.end(), items.begin() + i * per_item, items.begin() + (i + k) * per_item);
    }
  };
  auto runs = [&](uint32_t op, const std::vector<uint32_t>& qs, uint32_t arity) {
    std::vector<uint32_t> items;
    ++stamp;
    for (size_t i = 0; i < qs.size(); i += arity) {
      bool clash = false;
      for (uint32_t j = 0; j < arity; ++j) clash |= seen[qs[i + j]] == stamp;
      if (clash) {
        emit(op, items, 1);
        items.clear();
        ++stamp;
      }
      for (uint32_t j = 0; j < arity; ++j) seen[qs[i + j]] = stamp;
      items.push_back(arity == 2 ? (qs[i] | qs[i + 1] << 16) : qs[i]);
    }
    emit(op, items, 1);
  };
  for (const Op& op : c.ops) {
    const auto& t = op.targets;
    switch (op.kind) {
      case OpKind::H: runs(D_H, t, 1); break;
      case OpKind::S: runs(D_S, t, 1); break;
      case OpKind::X: runs(D_PX, t, 1); break;
      case OpKind::Y: runs(D_PY, t, 1); break;
      case OpKind::Z: runs(D_PZ, t, 1); break;
      case OpKind::CX: runs(D_CX, t, 2); break;
      case OpKind::XERR: case OpKind::YERR: case OpKind::ZERR: case OpKind::DEP1: case OpKind::DEP2: {
        const uint32_t kind = op.kind == OpKind::XERR ? F_X : op.kind == OpKind::YERR ? F_Y :
                              op.kind == OpKind::ZERR ? F_Z : op.kind == OpKind::DEP1 ? F_DEP1 : F_DEP2;
        std::vector<uint32_t> items;
        const uint32_t ar = kind == F_DEP2 ? 2 : 1;
        for (size_t i = 0; i < t.size(); i += ar) {
          items.push_back(t[i] | (ar == 2 ? t[i + 1] << 14 : 0u) | kind << 28);
          P.max_vars += kind == F_DEP1 ? 2 : kind == F_DEP2 ? 4 : 1;
          ++P.n_locs;
        }
        emit(D_FAULT, items, 1);
        break;
      }
      case OpKind::M: case OpKind::R: case OpKind::MR: {
        emit(op.kind == OpKind::M ? D_M : op.kind == OpKind::R ? D_R : D_MR, t, 1);
        if (op.kind != OpKind::R) P.list_bound += P.max_vars * t.size();
        P.max_vars += t.size();
        P.n_locs += (uint32_t)t.size();
        if (op.kind != OpKind::R) P.n_rec += (uint32_t)t.size();
        break;
      }
      case OpKind::FX: case OpKind::FY: case OpKind::FZ: {
        const uint32_t pauli = op.kind == OpKind::FX ? 1 : op.kind == OpKind::FY ? 2 : 3;
        std::vector<uint32_t> items;
        for (size_t i = 0; i < t.size(); i += 2) {
          if (t[i] >= P.n_rec) throw sp::Error(SP_E_INVALID, "a Pauli is controlled by a later measurement");
          items.push_back(t[i]);
          items.push_back(t[i + 1] | pauli << 16);
        }
        emit(D_FB, items, 2);
        break;
      }
      default: break;
    }
  }
  return P;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Log and snapshot words the logged pass can need at most (DW words per mask).
void log_bounds(const DevProgram& P, uint32_t DW, uint64_t* log_words, uint64_t* snap_words) {
  uint64_t lw = 0, sw = 0;
  for (size_t pc = 0; pc < P.words.size();) {
    const uint32_t hdr = P.words[pc], op = hdr & 0xFFu, cnt = hdr >> 8;
    if (op == D_FAULT) {
      const uint32_t kind = P.words[pc + 1] >> 28;
      lw += 3;
      sw += (uint64_t)cnt * (kind == F_DEP2 ? 2u : 1u) * 2u * DW;
    } else if (op == D_M || op == D_R || op == D_MR) {
      lw += (uint64_t)cnt * (3 + 2ull * DW);   // an entry each, and at most one RUN entry each
    } else if (op == D_FB) {
      lw += (uint64_t)cnt * (2 + (uint64_t)DW);
    }
    pc += 1 + (size_t)cnt * (op == D_FB ? 2u : 1u);
  }
  *log_words = lw;
  *snap_words = sw;
}

struct InitLayout {
  size_t ops, X, Z, P, E, loc, rec_var, rec_off, rec_len, rec_c, rec_det, status, log, snap, first, list, total;
  uint32_t RW, W, DW, list_cap;
};

// The buffer layout.  One pass: the index list takes whatever the buffer has
// left (at least `tail` entries).  Two passes (no phase rows here): the log,
// the snapshots and the first-entry table of the variable words, then
// `tail` bytes for the rows of E, the list counts and offsets and the
// lists, or whatever the buffer has left.
InitLayout layout(const sp_circuit& c, const DevProgram& P, bool two_pass, size_t tail, size_t budget) {
  InitLayout L{};
  const uint32_t n = c.n_qubits;
  L.RW = std::max<uint32_t>(1, (2 * n + 63) / 64);
  L.W = (uint32_t)std::max<uint64_t>(1, (P.max_vars + 64) / 64);
  L.DW = std::max<uint32_t>(1, (n + 63) / 64);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 1));
    return o;
  };
  L.ops = take(4 * P.words.size());
  L.X = take(8ull * n * L.RW);
  L.Z = take(8ull * n * L.RW);
  if (!two_pass) {
    L.P = take(8ull * n * L.W);
    L.E = take(16ull * L.W);
  }
  L.loc = take(4ull * P.n_locs);
  L.rec_var = take(4ull * P.n_rec);
  L.rec_off = take(4ull * P.n_rec);
  L.rec_len = take(4ull * P.n_rec);
  L.rec_c = take(4ull * P.n_rec);
  L.rec_det = take(4ull * P.n_rec);
  L.status = take(64);
  if (two_pass) {
    uint64_t lw = 0, sw = 0;
    log_bounds(P, L.DW, &lw, &sw);
    L.log = take(8 * lw);
    L.snap = take(8 * sw);
    L.first = take(8ull * L.W);   // zeroed with the rest of the fixed part
  }
  L.list = off;   // one pass: the lists; two passes: the rows of E and what follows them
  const size_t unit = two_pass ? 1 : 4;
  size_t room = tail;
  if (budget > off + unit * tail) room = std::min<size_t>((budget - off) / unit, two_pass ? SIZE_MAX : 0xFFFFFFFFull);
  L.list_cap = (uint32_t)std::min<size_t>(room, 0xFFFFFFFFull);
  L.total = align256(off + unit * room);
  return L;
}

// Default room after the fixed part.  One pass: index-list entries (the
// bound, at most 2^26).  Two passes: bytes for the rows of E of every
// recorded outcome and their lists, at most 1 GiB; a call that needs more
// says how much.
size_t default_tail(const DevProgram& P, bool two_pass) {
  if (!two_pass) return (size_t)std::min<uint64_t>(P.list_bound, 1ull << 26);
  const uint64_t W = std::max<uint64_t>(1, (P.max_vars + 64) / 64);
  const uint64_t need = (uint64_t)P.n_rec * (8 * W + 8) + 4 * std::min<uint64_t>(P.list_bound, 1ull << 26) + 1024;
  return (size_t)std::min<uint64_t>(need, 1ull << 30);
}

// Two passes pay unless the phase rows are small: the one-pass kernel
// updates them from one CU, the replay from every CU, and the logged pass
// takes runs of determined outcomes together.  Measured end to end: surface
// d=7 (122 KB of rows) 2.6 ms one pass, 1.4 ms two; d=15 (5.7 MB) 31 and 10
// ms; layered random 3c n=100 (252 KB) 3.9 and 3.5 ms; below 64 KB the
// random-outcome-heavy circuits (3a/3b n = 60-200, 2-52 KB) are 5-25%
// faster in one pass.
bool pick_two_pass(const sp_circuit& c, const DevProgram& P, int mode) {
  if (mode == SP_INIT_ONE_PASS) return false;
  if (mode == SP_INIT_TWO_PASS) return true;
  const uint64_t W = (P.max_vars + 64) / 64;
  return (uint64_t)c.n_qubits * W * 8 > (64ull << 10);
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return set_error(SP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int check_circuit(const sp_circuit* c) {
  if (c->n_qubits > kMaxQubits)
    return set_error(SP_E_LIMIT, "device Initialization supports up to " + std::to_string(kMaxQubits) + " qubits");
  return SP_OK;
}

// Launches the tableau pass (one or logged), the tableau in LDS when it fits.
template <bool LOG>
int launch_init(const InitDev& d, uint32_t n, uint32_t RW, hipStream_t s) {
  int dev = 0, lds_max = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const size_t tab_bytes = 16ull * n * RW;
  if (tab_bytes + kStaticLds <= (size_t)lds_max) {
    if (tab_bytes > 64 * 1024)
      HIP_TRY(hipFuncSetAttribute((const void*)init_kernel<true, LOG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)tab_bytes));
    hipLaunchKernelGGL((init_kernel<true, LOG>), dim3(1), dim3(kThreads), tab_bytes, s, d);
  } else {
    hipLaunchKernelGGL((init_kernel<false, LOG>), dim3(1), dim3(kThreads), 0, s, d);
  }
  HIP_TRY(hipGetLastError());
  return SP_OK;
}

// *need: a work-buffer size that suffices, when the call fails because the
// buffer is too small (SP_E_INVALID for the fixed part, SP_E_LIMIT for the
// lists); left 0 otherwise.
int symbolize_device(const sp_circuit& c, int outputs, int mode, void* d_work, size_t work_bytes, hipStream_t s,
                     sp_model** out, size_t* need) {
  const DevProgram P = compile(c);
  if (P.max_vars >= (1ull << 24)) return set_error(SP_E_LIMIT, "more than 2^24 variables");
  if (P.n_locs != c.n_locs || P.n_rec != c.n_meas) return set_error(SP_E_INVALID, "inconsistent circuit");
  const bool two = pick_two_pass(c, P, mode);
  const InitLayout L = layout(c, P, two, 0, work_bytes);
  if (L.total > work_bytes) {
    *need = L.total;
    return set_error(SP_E_INVALID, "work buffer of " + std::to_string(work_bytes) + " bytes, need at least " +
                                       std::to_string(L.total));
  }
  uint8_t* base = (uint8_t*)d_work;
  HIP_TRY(hipMemsetAsync(base, 0, L.list, s));
  if (!P.words.empty()) HIP_TRY(hipMemcpyAsync(base + L.ops, P.words.data(), 4 * P.words.size(), hipMemcpyHostToDevice, s));
  InitDev d{};
  d.ops = (const uint32_t*)(base + L.ops);
  d.n_words = (uint32_t)P.words.size();
  d.n = c.n_qubits;
  d.RW = L.RW;
  d.W = L.W;
  d.X = (uint64_t*)(base + L.X);
  d.Z = (uint64_t*)(base + L.Z);
  d.loc_var0 = (int32_t*)(base + L.loc);
  d.rec_var = (int32_t*)(base + L.rec_var);
  d.rec_off = (uint32_t*)(base + L.rec_off);
  d.rec_len = (uint32_t*)(base + L.rec_len);
  d.rec_c = (uint32_t*)(base + L.rec_c);
  d.rec_det = (int32_t*)(base + L.rec_det);
  d.status = (uint32_t*)(base + L.status);
  if (two) {
    d.log = (uint64_t*)(base + L.log);
    d.snap = (uint64_t*)(base + L.snap);
    d.first = (uint64_t*)(base + L.first);
    if (int rc = launch_init<true>(d, c.n_qubits, L.RW, s)) return rc;
  } else {
    d.P = (uint64_t*)(base + L.P);
    d.E = (uint64_t*)(base + L.E);
    d.list = (uint32_t*)(base + L.list);
    d.list_cap = L.list_cap;
    if (int rc = launch_init<false>(d, c.n_qubits, L.RW, s)) return rc;
  }

  uint32_t status[11] = {};
  std::vector<int32_t> loc_var0(c.n_locs), rec_var(c.n_meas), rec_det(c.n_meas);
  std::vector<uint32_t> rec_off(c.n_meas), rec_len(c.n_meas), rec_c(c.n_meas);
  HIP_TRY(hipMemcpyAsync(status, d.status, sizeof status, hipMemcpyDeviceToHost, s));
  if (c.n_locs) HIP_TRY(hipMemcpyAsync(loc_var0.data(), d.loc_var0, 4ull * c.n_locs, hipMemcpyDeviceToHost, s));
  if (c.n_meas) {
    HIP_TRY(hipMemcpyAsync(rec_var.data(), d.rec_var, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rec_off.data(), d.rec_off, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rec_len.data(), d.rec_len, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rec_c.data(), d.rec_c, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
    if (two) HIP_TRY(hipMemcpyAsync(rec_det.data(), d.rec_det, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (status[4] != c.n_locs || status[5] != c.n_meas) return set_error(SP_E_DEVICE, "device Initialization incomplete");
  std::vector<uint32_t> list;

  if (!two) {
    if (status[3]) {
      *need = layout(c, P, false, (size_t)std::min<uint64_t>(P.list_bound, 0xFFFFFFFFull), 0).total;
      return set_error(SP_E_LIMIT, "determined outcomes need more index-list room than the work buffer has (" +
                                       std::to_string(L.list_cap) + " entries); at most " + std::to_string(*need) +
                                       " bytes suffice");
    }
    list.resize(status[2]);
    if (status[2]) {
      HIP_TRY(hipMemcpyAsync(list.data(), base + L.list, 4ull * status[2], hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
  } else {
    // Replay the log over the phase rows, a slice of K words per workgroup.
    const uint64_t log_words = (uint64_t)status[6] | (uint64_t)status[7] << 32;
    const uint32_t n_vars = status[0], n_det = status[10];
    const uint32_t Wu = std::max<uint32_t>(1, (n_vars + 63) / 64);   // words of the phase rows in use
    // After the fixed part: rows of E, then counts and offsets, then the lists.
    const size_t e_off = L.list, cnt_off = align256(e_off + 8ull * n_det * Wu), ofs_off = align256(cnt_off + 4ull * n_det);
    const size_t lst_off = align256(ofs_off + 4ull * n_det);
    if (lst_off > work_bytes) {
      // The lists' length is known only after the replay; their bound is
      // every determined outcome holding every variable.
      *need = align256(lst_off + 4 * std::min<uint64_t>(P.list_bound, (uint64_t)n_det * n_vars));
      return set_error(SP_E_LIMIT, "the replay needs a work buffer of at least " + std::to_string(lst_off) +
                                       " bytes plus room for the index lists; " + std::to_string(*need) +
                                       " bytes suffice");
    }
    uint64_t* E = (uint64_t*)(base + e_off);
    if (n_det) HIP_TRY(hipMemsetAsync(E, 0, 8ull * n_det * Wu, s));   // slices skip the entries before their variables
    if (log_words) {
      int dev = 0, lds_max = 0;
      HIP_TRY(hipGetDevice(&dev));
      HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      const size_t n = std::max<uint32_t>(c.n_qubits, 1);
      const uint32_t K = (uint32_t)std::max<size_t>(1, std::min<size_t>(64, ((size_t)lds_max - kReplayStaticLds) / (8 * n)));
      ReplayArgs ra{};
      ra.log = d.log;
      ra.log_words = log_words;
      ra.snap = d.snap;
      ra.first = d.first;
      ra.E = E;
      ra.n = c.n_qubits;
      ra.DW = L.DW;
      ra.K = K;
      ra.W = Wu;
      const size_t lds = 8 * n * K;
      if (lds > 64 * 1024)
        HIP_TRY(hipFuncSetAttribute((const void*)replay_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL(replay_kernel, dim3((Wu + K - 1) / K), dim3(kReplayThreads), lds, s, ra);
      HIP_TRY(hipGetLastError());
    }
    // Lists of the determined recorded outcomes.
    std::vector<uint32_t> counts(n_det), offsets(n_det);
    if (n_det) {
      uint32_t* d_counts = (uint32_t*)(base + cnt_off);
      uint32_t* d_offsets = (uint32_t*)(base + ofs_off);
      hipLaunchKernelGGL(count_kernel, dim3(n_det), dim3(kListThreads), 0, s, (const uint64_t*)E, Wu, d_counts);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(counts.data(), d_counts, 4ull * n_det, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      uint64_t total = 0;
      for (uint32_t i = 0; i < n_det; ++i) {
        offsets[i] = (uint32_t)total;
        total += counts[i];
        if (total > 0xFFFFFFFFull) return set_error(SP_E_LIMIT, "more than 2^32 list entries");
      }
      if (lst_off + 4 * total > work_bytes) {
        *need = align256(lst_off + 4 * total);
        return set_error(SP_E_LIMIT, "the replay needs a work buffer of at least " + std::to_string(*need) +
                                         " bytes");
      }
      list.resize(total);
      if (total) {
        HIP_TRY(hipMemcpyAsync(d_offsets, offsets.data(), 4ull * n_det, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(write_lists_kernel, dim3(n_det), dim3(kListThreads), 0, s, (const uint64_t*)E, Wu,
                           (const uint32_t*)d_offsets, (uint32_t*)(base + lst_off));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(list.data(), base + lst_off, 4ull * total, hipMemcpyDeviceToHost, s));
      }
      HIP_TRY(hipStreamSynchronize(s));
    }
    for (uint32_t k = 0; k < c.n_meas; ++k)
      if (rec_var[k] < 0) {
        if (rec_det[k] < 0 || (uint32_t)rec_det[k] >= n_det) return set_error(SP_E_DEVICE, "bad outcome record");
        rec_off[k] = offsets[rec_det[k]];
        rec_len[k] = counts[rec_det[k]];
      }
  }

  std::vector<sp::Expr> outcomes(c.n_meas);
  for (uint32_t k = 0; k < c.n_meas; ++k) {
    sp::Expr& e = outcomes[k];
    if (rec_var[k] >= 0) {
      e.v.assign(1, (uint32_t)rec_var[k]);
    } else {
      e.c = (uint8_t)(rec_c[k] & 1u);
      if ((uint64_t)rec_off[k] + rec_len[k] > list.size()) return set_error(SP_E_DEVICE, "bad outcome list");
      e.v.assign(list.begin() + rec_off[k], list.begin() + rec_off[k] + rec_len[k]);
    }
  }
  *out = sp::assemble_model(c, outputs, std::move(loc_var0), status[0], status[1], outcomes);
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_symbolize_device_work_bytes_mode(const sp_circuit* circuit, int mode, size_t* bytes) {
  if (!circuit || !bytes) return set_error(SP_E_INVALID, "null argument");
  if (mode < SP_INIT_AUTO || mode > SP_INIT_TWO_PASS) return set_error(SP_E_INVALID, "unknown mode");
  if (int rc = check_circuit(circuit)) return rc;
  try {
    const DevProgram P = compile(*circuit);
    const bool two = pick_two_pass(*circuit, P, mode);
    *bytes = layout(*circuit, P, two, default_tail(P, two), 0).total;
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  return SP_OK;
}

int sp_symbolize_device_work_bytes(const sp_circuit* circuit, size_t* bytes) {
  return sp_symbolize_device_work_bytes_mode(circuit, SP_INIT_AUTO, bytes);
}

int sp_symbolize_device_mode(const sp_circuit* circuit, int outputs, int mode, void* d_work, size_t work_bytes,
                             void* stream, sp_model** out, size_t* need_bytes) {
  size_t need = 0;
  if (need_bytes) *need_bytes = 0;
  if (!circuit || !out || !d_work) return set_error(SP_E_INVALID, "null argument");
  *out = nullptr;
  if (outputs != SP_OUT_MEASUREMENTS && outputs != SP_OUT_DETECTORS)
    return set_error(SP_E_INVALID, "unknown outputs " + std::to_string(outputs));
  if (mode < SP_INIT_AUTO || mode > SP_INIT_TWO_PASS) return set_error(SP_E_INVALID, "unknown mode");
  if (((uintptr_t)d_work & 255u) != 0) return set_error(SP_E_INVALID, "work buffer must be 256-byte aligned");
  if (int rc = check_circuit(circuit)) return rc;
  try {
    const int rc = symbolize_device(*circuit, outputs, mode, d_work, work_bytes, (hipStream_t)stream, out, &need);
    if (need_bytes) *need_bytes = need;
    return rc;
  } catch (const sp::Error& e) {
    return set_error(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
}

int sp_symbolize_device(const sp_circuit* circuit, int outputs, void* d_work, size_t work_bytes, void* stream,
                        sp_model** out) {
  return sp_symbolize_device_mode(circuit, outputs, SP_INIT_AUTO, d_work, work_bytes, stream, out, nullptr);
}

}  // extern "C"

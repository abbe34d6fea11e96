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
//   E     the expression of the latest determined measurement (W words).
// Destabilizer phases are never read (as on the host).
//
// Init-P: the fault variable j on qubit q adds s_j to the stabilizer rows
// it anticommutes with.  A fault instruction's variables are consecutive, so
// each wave takes a 64-variable word of P: every lane gathers its variable's
// column word (z_q for X, x_q for Z) and 64 ballots transpose the 64x64 bit
// block into the 64 rows' words.
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
constexpr uint32_t kMaxQubits = 1024;
constexpr uint32_t kMaxRW = 2 * kMaxQubits / 64;   // 32
constexpr uint32_t kChunks = 32;                   // column chunks of the random-branch g sums

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
  uint32_t* status;     // n_vars, n_random, list used, overflow, n_locs, n_rec
};

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

// A vector load of memory this kernel writes, also where the address is
// uniform (a scalar-cache load would not see the workgroup's own stores).
template <class T>
__device__ __forceinline__ T ld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__global__ void __launch_bounds__(kThreads) init_kernel(InitDev d) {
  __shared__ uint64_t s_C[kMaxRW];      // constant phase bit of every row
  __shared__ uint64_t s_mask[kMaxRW];
  __shared__ uint64_t s_t[kMaxRW];
  __shared__ uint64_t s_c0[kMaxRW * kChunks];
  __shared__ uint64_t s_c1[kMaxRW * kChunks];
  __shared__ uint32_t s_rows[kMaxQubits];
  __shared__ uint32_t s_scan[kThreads / 64];
  __shared__ uint32_t s_u32[4];

  const uint32_t tid = threadIdx.x;
  const uint32_t n = d.n, RW = d.RW, W = d.W;

  // |0...0>: destabilizer i = X_i, stabilizer i = Z_i (buffers arrive zeroed).
  if (tid < kMaxRW) s_C[tid] = 0;
  for (uint32_t q = tid; q < n; q += kThreads) {
    d.X[(size_t)q * RW + (q >> 6)] |= 1ull << (q & 63);
    d.Z[(size_t)q * RW + ((n + q) >> 6)] |= 1ull << ((n + q) & 63);
  }
  __syncthreads();

  uint32_t vars = 0, n_random = 0, nloc = 0, nrec = 0, listu = 0, overflow = 0;

  // Rows of s_mask (its stabilizer or its destabilizer part) into s_rows,
  // ascending; returns the count.  One wave: lane l places bit l of each word.
  auto list_rows = [&](bool stab) -> uint32_t {
    if (tid < 64) {
      uint32_t cnt = 0;
      for (uint32_t w = 0; w < RW; ++w) {
        const uint64_t m = s_mask[w] & (stab ? stab_mask(w, n) : destab_mask(w, n));
        if ((m >> tid) & 1u) s_rows[cnt + (uint32_t)__builtin_popcountll(m & ((1ull << tid) - 1))] = w * 64 + tid;
        cnt += (uint32_t)__builtin_popcountll(m);
      }
      if (tid == 0) s_u32[1] = cnt;
    }
    __syncthreads();
    return uni(s_u32[1]);
  };

  // X^(px e) Z^(pz e) on qubit q for an outcome expression e: adds e to the
  // stabilizer rows the Pauli anticommutes with (Fact 1 with a vector
  // exponent).  e is the single variable e_var, or (e_var < 0) the first Wt
  // words of E, plus the constant e_c.
  auto add_expr = [&](uint32_t q, uint32_t px, uint32_t pz, int32_t e_var, uint32_t e_c, uint32_t Wt) {
    if (tid < RW)
      s_mask[tid] = ((px ? d.Z[(size_t)q * RW + tid] : 0ull) ^ (pz ? d.X[(size_t)q * RW + tid] : 0ull)) &
                    stab_mask(tid, n);
    __syncthreads();
    const uint32_t nr = list_rows(true);
    if (e_var >= 0) {
      for (uint32_t i = tid; i < nr; i += kThreads)
        d.P[(size_t)(s_rows[i] - n) * W + ((uint32_t)e_var >> 6)] ^= 1ull << ((uint32_t)e_var & 63);
    } else {
      for (uint32_t i = tid; i < nr * Wt; i += kThreads) {
        const uint32_t r = s_rows[i / Wt], w = i % Wt;
        d.P[(size_t)(r - n) * W + w] ^= d.E[w];
      }
    }
    if (e_c && tid < RW) s_C[tid] ^= s_mask[tid];
    __syncthreads();
  };

  for (uint32_t pc = 0; pc < d.n_words;) {
    const uint32_t hdr = uni(d.ops[pc]);
    const uint32_t op = hdr & 0xFFu, cnt = hdr >> 8;
    const uint32_t* it = d.ops + pc + 1;
    pc += 1 + cnt * (op == D_FB ? 2u : 1u);

    if (op == D_H || op == D_S || op == D_PX || op == D_PY || op == D_PZ || op == D_CX) {
      for (uint32_t i = tid; i < cnt * RW; i += kThreads) {
        const uint32_t k = i / RW, w = i % RW;
        const uint32_t item = it[k];
        if (op == D_CX) {
          const uint32_t a = item & 0xFFFFu, b = item >> 16;
          uint64_t& xa = d.X[(size_t)a * RW + w];
          uint64_t& za = d.Z[(size_t)a * RW + w];
          uint64_t& xb = d.X[(size_t)b * RW + w];
          uint64_t& zb = d.Z[(size_t)b * RW + w];
          const uint64_t vxa = xa, vza = za, vxb = xb, vzb = zb;
          const uint64_t t = vxa & vzb & ~(vxb ^ vza);
          if (t) atomicXor((unsigned long long*)&s_C[w], (unsigned long long)t);
          xb = vxb ^ vxa;
          za = vza ^ vzb;
        } else {
          uint64_t& x = d.X[(size_t)item * RW + w];
          uint64_t& z = d.Z[(size_t)item * RW + w];
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
      // 64*vw + l, gathers the column word that decides which stabilizer
      // rows anticommute with its Pauli (z_q for X, x_q for Z, both for Y),
      // and 64 ballots transpose that word: ballot j is row 64*w + j's
      // bits for the wave's 64 variables, kept by lane j.
      const uint32_t lane = tid & 63u;
      const uint32_t vw0 = vars >> 6, vw1 = (vars + nv - 1) >> 6;
      const uint32_t sw0 = n >> 6, sw1 = (2 * n - 1) >> 6;
      for (uint32_t vw = vw0 + (tid >> 6); vw <= vw1; vw += kThreads / 64) {
        const uint32_t v = vw * 64 + lane;
        const uint64_t* col_z = nullptr;
        const uint64_t* col_x = nullptr;
        if (v >= vars && v < vars + nv) {
          const uint32_t rel = v - vars, item = it[rel >> lg], b = rel & ((1u << lg) - 1u);
          const uint32_t kind = item >> 28;
          const uint32_t q = b >= 2 ? (item >> 14) & 0x3FFFu : item & 0x3FFFu;
          const bool xf = kind == F_X || kind == F_Y || ((kind == F_DEP1 || kind == F_DEP2) && !(b & 1u));
          const bool zf = kind == F_Z || kind == F_Y || ((kind == F_DEP1 || kind == F_DEP2) && (b & 1u));
          if (xf) col_z = d.Z + (size_t)q * RW;
          if (zf) col_x = d.X + (size_t)q * RW;
        }
        for (uint32_t w = sw0; w <= sw1; ++w) {
          uint64_t col = 0;
          if (col_z) col ^= col_z[w];
          if (col_x) col ^= col_x[w];
          col &= stab_mask(w, n);
          if (__ballot(col != 0) == 0) continue;
          uint64_t out = 0;
#pragma unroll 16
          for (uint32_t j = 0; j < 64; ++j) {
            const uint64_t bal = __ballot((col >> j) & 1u);
            out = lane == j ? bal : out;
          }
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

    // Outcome records written by one thread are read by all below.
    __syncthreads();

    if (op == D_FB) {
      for (uint32_t k = 0; k < cnt; ++k) {
        const uint32_t rec = uni(it[2 * k]), qp = uni(it[2 * k + 1]);
        const uint32_t q = qp & 0xFFFFu, pauli = qp >> 16;   // 1 X, 2 Y, 3 Z
        const uint32_t px = pauli != 3, pz = pauli != 1;
        const int32_t rv = (int32_t)uni((uint32_t)ld(d.rec_var + rec));
        const uint32_t ec = uni(ld(d.rec_c + rec));
        const uint32_t off = uni(ld(d.rec_off + rec)), len = uni(ld(d.rec_len + rec));
        const uint32_t Wt = (vars + 63) >> 6;
        if (rv < 0) {
          // E <- the recorded list as a dense row; the first entry of each
          // word gathers that word's entries (the list is ascending).
          for (uint32_t w = tid; w < Wt; w += kThreads) d.E[w] = 0;
          __syncthreads();
          for (uint32_t i = tid; i < len; i += kThreads) {
            const uint32_t s0 = ld(d.list + off + i), w = s0 >> 6;
            if (i == 0 || (ld(d.list + off + i - 1) >> 6) != w) {
              uint64_t e = 0;
              for (uint32_t j = i; j < len; ++j) {
                const uint32_t sj = ld(d.list + off + j);
                if ((sj >> 6) != w) break;
                e |= 1ull << (sj & 63);
              }
              d.E[w] = e;
            }
          }
          __syncthreads();
        }
        add_expr(q, px, pz, rv, ec, Wt);
      }
      continue;
    }

    // D_M, D_R, D_MR: one location per target, in order.
    for (uint32_t k = 0; k < cnt; ++k) {
      const uint32_t a = uni(it[k]);
      const uint64_t* xa = d.X + (size_t)a * RW;
      if (tid == 0) s_u32[0] = 0xFFFFFFFFu;
      __syncthreads();
      if (tid < RW) {
        const uint64_t m = xa[tid] & stab_mask(tid, n);
        if (m) atomicMin(&s_u32[0], tid * 64 + (uint32_t)__builtin_ctzll(m));
      }
      __syncthreads();
      const uint32_t p = uni(s_u32[0]);
      int32_t e_var = -1;
      uint32_t e_c = 0;
      const uint32_t Wt = (vars + 1 + 63) >> 6;   // words holding every variable so far, and one more

      if (p != 0xFFFFFFFFu) {
        // ---- random outcome: a fresh variable -----------------------------
        e_var = (int32_t)vars;
        if (tid == 0) d.loc_var0[nloc] = (int32_t)vars;
        ++vars;
        ++n_random;
        if (tid < RW) s_mask[tid] = xa[tid] & ~(tid == (p >> 6) ? (1ull << (p & 63)) : 0ull);
        __syncthreads();
        // g sums of every row against row p, bit-sliced mod 4, per (word, column chunk).
        {
          const uint32_t w = tid % kMaxRW, chunk = tid / kMaxRW;
          if (w < RW) {
            uint64_t c0 = 0, c1 = 0;
            const uint64_t mw = s_mask[w];
            if (mw) {
              for (uint32_t q = chunk; q < n; q += kChunks) {
                const uint64_t* xq = d.X + (size_t)q * RW;
                const uint64_t* zq = d.Z + (size_t)q * RW;
                const uint64_t lx = bit_of(xq, p) ? ~0ull : 0ull, lz = bit_of(zq, p) ? ~0ull : 0ull;
                if (!(lx | lz)) continue;
                uint64_t plus, minus;
                g_masks(lx, lz, xq[w], zq[w], plus, minus);
                // c += plus; c -= minus (mod 4, per bit)
                c1 ^= c0 & plus;
                c0 ^= plus;
                c1 ^= ~c0 & minus;
                c0 ^= minus;
              }
            }
            s_c0[w * kChunks + chunk] = c0;
            s_c1[w * kChunks + chunk] = c1;
          }
        }
        __syncthreads();
        if (tid < RW) {
          uint64_t c0 = 0, c1 = 0;
          for (uint32_t ch = 0; ch < kChunks; ++ch) {
            const uint64_t b0 = s_c0[tid * kChunks + ch], b1 = s_c1[tid * kChunks + ch];
            c1 ^= b1 ^ (c0 & b0);
            c0 ^= b0;
          }
          s_t[tid] = c1;   // the sums are even for commuting rows: bit 1 says "2 mod 4"
        }
        const uint32_t cp = bit_of(s_C, p);
        const uint32_t nrows = list_rows(true);   // stabilizer rows taking row p (also syncs s_t)
        // Constants, then symbols of the stabilizer rows, then x/z of every row.
        if (tid < RW) {
          const uint64_t m = s_mask[tid] & stab_mask(tid, n);
          s_C[tid] ^= m & (s_t[tid] ^ (cp ? ~0ull : 0ull));
        }
        {
          const uint64_t* pp = d.P + (size_t)(p - n) * W;
          for (uint32_t i = tid; i < nrows * Wt; i += kThreads) {
            const uint32_t r = s_rows[i / Wt], w = i % Wt;
            d.P[(size_t)(r - n) * W + w] ^= pp[w];
          }
        }
        for (uint32_t i = tid; i < n * RW; i += kThreads) {
          const uint32_t q = i / RW, w = i % RW;
          uint64_t* xq = d.X + (size_t)q * RW;
          uint64_t* zq = d.Z + (size_t)q * RW;
          const uint64_t lx = bit_of(xq, p) ? ~0ull : 0ull, lz = bit_of(zq, p) ? ~0ull : 0ull;
          xq[w] ^= s_mask[w] & lx;
          zq[w] ^= s_mask[w] & lz;
        }
        __syncthreads();
        // Destabilizer p-n <- row p; row p <- Z_a with phase +s_var.
        for (uint32_t q = tid; q < n; q += kThreads) {
          uint64_t* xq = d.X + (size_t)q * RW;
          uint64_t* zq = d.Z + (size_t)q * RW;
          const uint32_t bx = bit_of(xq, p), bz = bit_of(zq, p);
          const uint32_t dr = p - n;
          xq[dr >> 6] = (xq[dr >> 6] & ~(1ull << (dr & 63))) | ((uint64_t)bx << (dr & 63));
          zq[dr >> 6] = (zq[dr >> 6] & ~(1ull << (dr & 63))) | ((uint64_t)bz << (dr & 63));
          xq[p >> 6] &= ~(1ull << (p & 63));
          zq[p >> 6] = (zq[p >> 6] & ~(1ull << (p & 63))) | ((q == a ? 1ull : 0ull) << (p & 63));
        }
        if (tid == 0) s_C[p >> 6] &= ~(1ull << (p & 63));
        {
          uint64_t* pp = d.P + (size_t)(p - n) * W;
          const uint32_t Wn = (vars + 63) >> 6;
          for (uint32_t w = tid; w < Wn; w += kThreads)
            pp[w] = (w == ((uint32_t)e_var >> 6)) ? (1ull << ((uint32_t)e_var & 63)) : 0ull;
        }
        __syncthreads();
      } else {
        // ---- determined outcome --------------------------------------------
        if (tid == 0) d.loc_var0[nloc] = -1;
        if (tid < RW) s_mask[tid] = xa[tid] & destab_mask(tid, n);
        __syncthreads();
        const uint32_t ns = list_rows(false);   // destabilizer rows i: the product takes stabilizer n+i
        // g sums, column by column, of the ordered product into the scratch row.
        uint32_t g = 0;
        for (uint32_t q = tid; q < n; q += kThreads) {
          const uint64_t* xq = d.X + (size_t)q * RW;
          const uint64_t* zq = d.Z + (size_t)q * RW;
          uint32_t xs = 0, zs = 0;
          for (uint32_t j = 0; j < ns; ++j) {
            const uint32_t r = n + s_rows[j];
            const uint32_t xi = bit_of(xq, r), zi = bit_of(zq, r);
            uint64_t plus, minus;
            g_masks(xi ? 1ull : 0ull, zi ? 1ull : 0ull, xs, zs, plus, minus);
            g += (uint32_t)plus - (uint32_t)minus;   // mod 2^32, reduced mod 4 below
            xs ^= xi;
            zs ^= zi;
          }
        }
        // Constant: the selected stabilizers' constants and the g correction.
        uint32_t cpar = 0;
        for (uint32_t j = tid; j < ns; j += kThreads) cpar ^= bit_of(s_C, n + s_rows[j]);
        if (tid == 0) {
          s_u32[2] = 0;
          s_u32[3] = 0;
        }
        __syncthreads();
        if (g & 3u) atomicAdd(&s_u32[2], g & 3u);
        if (cpar) atomicXor(&s_u32[3], 1u);
        // Symbols: E = XOR of the selected stabilizers' P rows.
        for (uint32_t w = tid; w < Wt; w += kThreads) {
          uint64_t e = 0;
          for (uint32_t j = 0; j < ns; ++j) e ^= d.P[(size_t)s_rows[j] * W + w];
          d.E[w] = e;
        }
        __syncthreads();
        e_c = uni(s_u32[3]) ^ (((uni(s_u32[2]) & 3u) == 2u) ? 1u : 0u);
      }

      // Record the outcome (M, MR).
      if (op != D_R) {
        if (e_var >= 0) {
          if (tid == 0) {
            d.rec_var[nrec] = e_var;
            d.rec_c[nrec] = 0;
            d.rec_off[nrec] = 0;
            d.rec_len[nrec] = 0;
          }
        } else {
          // Sorted list of E's set bits: per-thread word ranges, a block scan.
          const uint32_t per = (Wt + kThreads - 1) / kThreads;
          const uint32_t w0 = tid * per, w1 = min(Wt, w0 + per);
          uint32_t mine = 0;
          for (uint32_t w = w0; w < w1; ++w) mine += (uint32_t)__builtin_popcountll(d.E[w]);
          // Exclusive scan of the counts: within each wave by shuffles, then
          // over the waves' totals.
          const uint32_t lane = tid & 63u, wave = tid >> 6;
          uint32_t incl = mine;
          for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
          }
          if (lane == 63) s_scan[wave] = incl;
          __syncthreads();
          uint32_t before = 0, total = 0;
          for (uint32_t k = 0; k < kThreads / 64; ++k) {
            const uint32_t t = s_scan[k];
            before += k < wave ? t : 0u;
            total += t;
          }
          total = uni(total);
          const uint32_t fits = (uint64_t)listu + total <= d.list_cap;
          if (fits) {
            uint32_t pos = listu + before + incl - mine;
            for (uint32_t w = w0; w < w1; ++w) {
              uint64_t e = d.E[w];
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
          __syncthreads();
        }
        ++nrec;
      }
      // Reset (R, MR): X^e on qubit a.
      if (op != D_M) add_expr(a, 1, 0, e_var, e_c, Wt);
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

struct InitLayout {
  size_t ops, X, Z, P, E, loc, rec_var, rec_off, rec_len, rec_c, status, list, total;
  uint32_t RW, W, list_cap;
};

// The buffer layout; the index list takes whatever the buffer has left
// (at least list_min entries).
InitLayout layout(const sp_circuit& c, const DevProgram& P, size_t list_min, size_t budget) {
  InitLayout L{};
  const uint32_t n = c.n_qubits;
  L.RW = std::max<uint32_t>(1, (2 * n + 63) / 64);
  L.W = (uint32_t)std::max<uint64_t>(1, (P.max_vars + 64) / 64);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 1));
    return o;
  };
  L.ops = take(4 * P.words.size());
  L.X = take(8ull * n * L.RW);
  L.Z = take(8ull * n * L.RW);
  L.P = take(8ull * n * L.W);
  L.E = take(8ull * L.W);
  L.loc = take(4ull * P.n_locs);
  L.rec_var = take(4ull * P.n_rec);
  L.rec_off = take(4ull * P.n_rec);
  L.rec_len = take(4ull * P.n_rec);
  L.rec_c = take(4ull * P.n_rec);
  L.status = take(64);
  L.list = off;
  size_t cap = list_min;
  if (budget > off + 4 * list_min) cap = std::min<size_t>((budget - off) / 4, 0xFFFFFFFFull);
  L.list_cap = (uint32_t)cap;
  L.total = align256(off + 4 * cap);
  return L;
}

// Default index-list room: the bound, capped at 2^26 entries (256 MiB).
size_t default_list(const DevProgram& P) { return (size_t)std::min<uint64_t>(P.list_bound, 1ull << 26); }

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

}  // namespace

extern "C" {

int sp_symbolize_device_work_bytes(const sp_circuit* circuit, size_t* bytes) {
  if (!circuit || !bytes) return set_error(SP_E_INVALID, "null argument");
  if (int rc = check_circuit(circuit)) return rc;
  try {
    const DevProgram P = compile(*circuit);
    *bytes = layout(*circuit, P, default_list(P), 0).total;
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  return SP_OK;
}

int sp_symbolize_device(const sp_circuit* circuit, int outputs, void* d_work, size_t work_bytes, void* stream,
                        sp_model** out) {
  if (!circuit || !out || !d_work) return set_error(SP_E_INVALID, "null argument");
  *out = nullptr;
  if (outputs != SP_OUT_MEASUREMENTS && outputs != SP_OUT_DETECTORS)
    return set_error(SP_E_INVALID, "unknown outputs " + std::to_string(outputs));
  if (((uintptr_t)d_work & 255u) != 0) return set_error(SP_E_INVALID, "work buffer must be 256-byte aligned");
  if (int rc = check_circuit(circuit)) return rc;
  const sp_circuit& c = *circuit;
  try {
    const DevProgram P = compile(c);
    if (P.max_vars >= (1ull << 24)) return set_error(SP_E_LIMIT, "more than 2^24 variables");
    if (P.n_locs != c.n_locs || P.n_rec != c.n_meas) return set_error(SP_E_INVALID, "inconsistent circuit");
    const InitLayout L = layout(c, P, 0, work_bytes);
    if (L.total > work_bytes)
      return set_error(SP_E_INVALID, "work buffer of " + std::to_string(work_bytes) + " bytes, need at least " +
                                         std::to_string(L.total));
    hipStream_t s = (hipStream_t)stream;
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
    d.P = (uint64_t*)(base + L.P);
    d.E = (uint64_t*)(base + L.E);
    d.loc_var0 = (int32_t*)(base + L.loc);
    d.rec_var = (int32_t*)(base + L.rec_var);
    d.rec_off = (uint32_t*)(base + L.rec_off);
    d.rec_len = (uint32_t*)(base + L.rec_len);
    d.rec_c = (uint32_t*)(base + L.rec_c);
    d.list = (uint32_t*)(base + L.list);
    d.list_cap = L.list_cap;
    d.status = (uint32_t*)(base + L.status);
    hipLaunchKernelGGL(init_kernel, dim3(1), dim3(kThreads), 0, s, d);
    HIP_TRY(hipGetLastError());

    uint32_t status[6];
    std::vector<int32_t> loc_var0(c.n_locs), rec_var(c.n_meas);
    std::vector<uint32_t> rec_off(c.n_meas), rec_len(c.n_meas), rec_c(c.n_meas);
    HIP_TRY(hipMemcpyAsync(status, d.status, sizeof status, hipMemcpyDeviceToHost, s));
    if (c.n_locs) HIP_TRY(hipMemcpyAsync(loc_var0.data(), d.loc_var0, 4ull * c.n_locs, hipMemcpyDeviceToHost, s));
    if (c.n_meas) {
      HIP_TRY(hipMemcpyAsync(rec_var.data(), d.rec_var, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(rec_off.data(), d.rec_off, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(rec_len.data(), d.rec_len, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(rec_c.data(), d.rec_c, 4ull * c.n_meas, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (status[3])
      return set_error(SP_E_LIMIT, "determined outcomes need more index-list room than the work buffer has (" +
                                       std::to_string(L.list_cap) + " entries); at most " +
                                       std::to_string(layout(c, P, (size_t)std::min<uint64_t>(P.list_bound, 0xFFFFFFFFull), 0).total) +
                                       " bytes suffice");
    if (status[4] != c.n_locs || status[5] != c.n_meas) return set_error(SP_E_DEVICE, "device Initialization incomplete");
    std::vector<uint32_t> list(status[2]);
    if (status[2]) {
      HIP_TRY(hipMemcpyAsync(list.data(), d.list, 4ull * status[2], hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
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
  } catch (const sp::Error& e) {
    return set_error(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  return SP_OK;
}

}  // extern "C"

// Sampling of Algorithm 1 on gfx950: M_samples = M [b_1 ... b_nsmp] + c (Eq. 4).
//
// One workgroup owns one 64-shot word w: lane t of every wave stands for
// shot first_shot + 64 w + t.  The rows of the word's output column block
// (one uint64 per measurement) live in an LDS slab initialised from c.  The
// waves of the workgroup split the drawn locations between them, four
// locations (one Philox block) at a time:
//
//   draw     u = Philox4x32-10(ctr = (l/4, shot lo, shot hi, 0), key = seed)
//            -- the counter's first word and the key are wave-uniform, so
//               the compiler keeps the key schedule and the first rounds'
//               uniform products on the scalar unit;
//   select   fire = ballot(u < T_m): one compare per location gives the
//            64-lane mask of shots in which the location is not the identity
//            (all-zero in most words at p ~ 1e-3, and then nothing else runs);
//   decode   for depolarizing channels, masks m_k = ballot(u < T_k) are
//            nested, so code bit i is the XOR of the m_k at which bit i of
//            the code changes between k and k+1 -- pure scalar 64-bit XORs;
//   evaluate for every variable whose mask S is nonzero, XOR S into the slab
//            rows of its column of M (LDS atomics: ds_xor_b64), either from
//            the column list (sparse path) or from the n_m-bit column mask
//            (dense path);
//   store    after a barrier, slab row k goes to out[k*ld + w], with the
//            bits of shots past the end cleared.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device_model.hpp"

using sp::set_error;
using sp::DevModel;
using sp::LaunchArgs;
using sp::TileRec;
using sp::TiledArgs;
using sp::BatchJob;
using sp::BatchCounters;

namespace {

// Address-space views of model and output pointers.  The model is read-only
// while kernels run: uniform reads through the constant space become scalar
// loads, per-lane reads through the global space avoid flat instructions.
// (Pointers that come from a job table in memory would otherwise be generic.)
// The qualifiers mean something only to the device compiler.
#if defined(__HIP_DEVICE_COMPILE__)
#define SP_CONST_AS __attribute__((address_space(4)))
#define SP_GLOBAL_AS __attribute__((address_space(1)))
#else
#define SP_CONST_AS
#define SP_GLOBAL_AS
#endif
typedef const SP_CONST_AS uint32_t* cuint32_p;
typedef const SP_CONST_AS uint64_t* cuint64_p;
typedef const SP_GLOBAL_AS uint32_t* guint32_p;
typedef const SP_GLOBAL_AS uint64_t* guint64_p;
typedef const SP_GLOBAL_AS uint4* guint4_p;
typedef SP_GLOBAL_AS uint64_t* gout_p;

// A read-only object loaded through the constant space, 16 bytes at a time
// (wave-uniform address: scalar loads into SGPRs, merged by the compiler).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 16 == 0, "16-byte multiples only");
  T v;
  const SP_CONST_AS u32x4* src = (const SP_CONST_AS u32x4*)p;
  u32x4* dst = reinterpret_cast<u32x4*>(&v);
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 16; ++i) dst[i] = src[i];
  return v;
}

constexpr uint32_t kM0 = 0xD2511F53u;   // Philox4x32 round multipliers
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;   // Philox key increments
constexpr uint32_t kW1 = 0xBB67AE85u;

// Round keys of Philox4x32-10 for one seed: round r uses (key0 + r*W0,
// key1 + r*W1).  They are wave-uniform SGPR operands of each round's
// three-input XOR.
struct RoundKeys {
  uint32_t k0[10], k1[10];
};

// A uniform value held in a vector register.
__device__ __forceinline__ uint32_t to_vgpr(uint32_t x) {
  uint32_t v;
  asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
  return v;
}

__device__ __forceinline__ RoundKeys round_keys(uint32_t key0, uint32_t key1) {
  RoundKeys k;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    k.k0[r] = key0 + (uint32_t)r * kW0;
    k.k1[r] = key1 + (uint32_t)r * kW1;
  }
  return k;
}

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                             uint32_t k1) {
  const uint64_t p0 = (uint64_t)kM0 * c0;
  const uint64_t p1 = (uint64_t)kM1 * c2;
  // three-input XOR in one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
  const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
  const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
  c1 = (uint32_t)p1;
  c3 = (uint32_t)p0;
  c0 = n0;
  c2 = n2;
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// products on words 0 and 2, then (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
// the key advances by (W0, W1) between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               const RoundKeys& k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) philox_round(c0, c1, c2, c3, k.k0[r], k.k1[r]);
  return make_uint4(c0, c1, c2, c3);
}

// Scalar-unit arithmetic on wave-uniform words.  The compiler moves a
// uniform computation to the vector unit as soon as one operand sits in a
// vector register; these keep each step on the scalar unit (operands are
// read into scalar registers first when needed).
__device__ __forceinline__ uint32_t s_mulhi(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("s_mul_hi_u32 %0, %1, %2" : "=s"(r) : "s"(a), "s"(b));
  return r;
}
__device__ __forceinline__ uint32_t s_mullo(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("s_mul_i32 %0, %1, %2" : "=s"(r) : "s"(a), "s"(b));
  return r;
}
__device__ __forceinline__ uint32_t s_xor(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("s_xor_b32 %0, %1, %2" : "=s"(r) : "s"(a), "s"(b) : "scc");
  return r;
}

// The draws of one 64-shot word.  Lane t's counter is (l/4, shot lo, shot
// hi, 0): within a wave the block index l/4, the key and (UHI: when the 64
// shots share it) the high word are uniform, so of the cipher's first rounds
// only part depends on the lane, and of that part some does not depend on
// the block.  Per word, before the block loop:
//   a   = hi(M1 * hi) ^ lo ^ k0[0]     round 1's first output word (lane)
//   b   = M0 * a                       round 2's first product (lane)
//   p1l = lo(M1 * hi)                  round 1's second output word (uniform)
// Per block, round 1 and the uniform halves of rounds 2-4 run on the scalar
// unit, leaving 15 products and 17 XORs per lane instead of 20 and 20.
struct ShotWord {
  uint32_t lo, hi;       // the shot index's words (hi uniform when UHI)
  uint32_t a, bhi, blo;  // lane-invariant words of rounds 1-2 (UHI)
  uint32_t p1l;          // uniform (UHI)
};

template <bool UHI>
__device__ __forceinline__ ShotWord shot_word(uint64_t shot0, uint32_t lane, const RoundKeys& k) {
  ShotWord w{};
  if (UHI) {
    w.lo = (uint32_t)shot0 + lane;
    w.hi = s_xor((uint32_t)(shot0 >> 32), 0u);
    w.p1l = s_mullo(w.hi, kM1);
    w.a = s_xor(s_mulhi(w.hi, kM1), k.k0[0]) ^ w.lo;
    const uint64_t b = (uint64_t)kM0 * w.a;
    w.bhi = (uint32_t)(b >> 32);
    w.blo = (uint32_t)b;
  } else {
    const uint64_t shot = shot0 + lane;
    w.lo = (uint32_t)shot;
    w.hi = (uint32_t)(shot >> 32);
  }
  return w;
}

// Philox4x32-10 of counter (blk, w.lo, w.hi, 0): the same value as
// philox4x32_10, with the UHI split above.
template <bool UHI>
__device__ __forceinline__ uint4 draw4(uint32_t blk, const ShotWord& w, const RoundKeys& k) {
  if (!UHI) return philox4x32_10(blk, w.lo, w.hi, 0u, k);
  // round 1: (a, p1l, hi(M0 blk) ^ k1[0], lo(M0 blk))
  const uint32_t c2 = s_xor(s_mulhi(blk, kM0), k.k1[0]);
  const uint32_t c3 = s_mullo(blk, kM0);
  // round 2: (hi(M1 c2) ^ p1l ^ k0[1], lo(M1 c2), bhi ^ c3 ^ k1[1], blo)
  const uint32_t d0 = s_xor(s_xor(s_mulhi(c2, kM1), w.p1l), k.k0[1]);
  const uint32_t d1 = s_mullo(c2, kM1);
  const uint32_t d2 = w.bhi ^ s_xor(c3, k.k1[1]);
  // round 3: (hi(M1 d2) ^ d1 ^ k0[2], lo(M1 d2), hi(M0 d0) ^ blo ^ k1[2], lo(M0 d0))
  const uint64_t r1 = (uint64_t)kM1 * d2;
  uint32_t c0 = (uint32_t)(r1 >> 32) ^ s_xor(d1, k.k0[2]);
  uint32_t c1 = (uint32_t)r1;
  const uint32_t e2 = w.blo ^ s_xor(s_mulhi(d0, kM0), k.k1[2]);
  const uint32_t e3 = s_mullo(d0, kM0);
  // round 4: the last uniform word enters through a scalar XOR
  const uint64_t s0 = (uint64_t)kM0 * c0;
  const uint64_t s1 = (uint64_t)kM1 * e2;
  c0 = __builtin_amdgcn_bitop3_b32((uint32_t)(s1 >> 32), c1, k.k0[3], 0x96);
  c1 = (uint32_t)s1;
  uint32_t c2l = (uint32_t)(s0 >> 32) ^ s_xor(e3, k.k1[3]);
  uint32_t c3l = (uint32_t)s0;
#pragma unroll
  for (int r = 4; r < 10; ++r) philox_round(c0, c1, c2l, c3l, k.k0[r], k.k1[r]);
  return make_uint4(c0, c1, c2l, c3l);
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t pick(const uint4& v, int s) {
  return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}

// A 32-bit word of a read-only device array at a per-lane index, addressed
// as a uniform base plus a 32-bit byte offset (the arrays stay under 4 GiB).
__device__ __forceinline__ uint32_t ld32(const uint32_t* base, uint32_t idx) {
  return *(const SP_GLOBAL_AS uint32_t*)((const SP_GLOBAL_AS char*)base + (idx << 2));
}

// Pauli code of a fired draw u under channel ch1 - 1: the k with
// T_{k-1} <= u < T_k (T_0 = 0).  The channel row holds kind | m << 8, then
// T_1..T_{m-1}, then 0xFFFFFFFF; T_1..T_15 is thus nondecreasing and a
// binary search counts j = #{k : T_k <= u}, so code = j + 1.  A draw of
// u = 2^32 - 1 fires only when T_m = 2^32 (p = 1), and its code is m.
__device__ __forceinline__ uint32_t lane_code(const uint32_t* chans, uint32_t ch1, uint32_t u) {
  const uint32_t t = (ch1 - 1u) * 16u;
  uint32_t j = 0;
  j += (ld32(chans, t + j + 8) <= u) ? 8u : 0u;
  j += (ld32(chans, t + j + 4) <= u) ? 4u : 0u;
  j += (ld32(chans, t + j + 2) <= u) ? 2u : 0u;
  j += (ld32(chans, t + j + 1) <= u) ? 1u : 0u;
  return min(j + 1u, ld32(chans, t) >> 8);
}

// Code-bit masks of a fired location (fire = lanes with u < T_m): mask i
// holds the fired lanes whose code has bit i set.
struct Masks {
  uint64_t b0, b1, b2, b3;   // 64-lane masks of code bits 0..3
  uint32_t nbits;            // code bits of the channel: 1, 2 or 4
};

__device__ __forceinline__ Masks decode(const uint32_t* chans, uint32_t meta, uint32_t u, uint64_t fire,
                                        uint32_t lane) {
  const uint32_t m = ((const cuint32_p)chans)[((meta & 0xFFu) - 1u) * 16u] >> 8;   // uniform
  Masks r{fire, 0ull, 0ull, 0ull, 1u};   // one code: X/Y/Z errors and the random-measurement coin
  if (m > 1) {
    const bool f = (fire >> lane) & 1ull;
    const uint32_t code = lane_code(chans, meta & 0xFFu, u);
    r.nbits = m == 3 ? 2u : 4u;
    r.b0 = ballot(f && (code & 1u));
    r.b1 = ballot(f && (code & 2u));
    r.b2 = ballot(f && (code & 4u));
    r.b3 = ballot(f && (code & 8u));
  }
  return r;
}

// Evaluate a fired location: XOR its code-bit masks into the slab rows of
// its variables' columns of M.
// Words of a dense column's bitmap of its non-zero words (bit c of the
// bitmap: mask word c is not zero); the column stores the bitmap, then its
// mask words.
__device__ __forceinline__ uint32_t nz_words(uint32_t dense_words) { return (dense_words + 63u) >> 6; }

// Only the column's non-zero words are visited (the bitmap read with scalar
// loads), four at a time so that their loads are in flight together.
__device__ __forceinline__ void xor_dense(const DevModel& m, uint64_t* slab, uint32_t var, uint64_t s, uint32_t lane) {
  const uint32_t nzw = nz_words(m.dense_words);
  const cuint64_p col = (cuint64_p)m.dense + (size_t)var * (m.dense_words + nzw);
  const uint64_t lb = 1ull << lane;
  for (uint32_t k = 0; k < nzw; ++k) {
    uint64_t nz = col[k];
    while (nz) {
      uint32_t c[4];
      uint64_t bits[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c[i] = nz ? k * 64u + (uint32_t)__builtin_ctzll(nz) : 0xFFFFFFFFu;
        nz &= nz - 1;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) bits[i] = c[i] != 0xFFFFFFFFu ? col[nzw + c[i]] : 0ull;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (bits[i] & lb) atomicXor((unsigned long long*)&slab[c[i] * 64 + lane], (unsigned long long)s);
    }
  }
}

constexpr uint32_t kNoEntry = 0xFFFFFFFFu;

// The slab row named by entry e = row << 5 | bit: e >> 2 is its byte offset.
__device__ __forceinline__ uint64_t& row_of(uint64_t* slab, uint32_t e) {
  return *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(slab) + (e >> 2));
}

// Mask of the code bit named by entry e (low two bits) among the first NB.
// Written as masked XORs rather than selects: the uniform masks stay scalar
// operands and no lookup table is formed.
template <int NB>
__device__ __forceinline__ uint64_t select_mask(uint32_t e, const Masks& k) {
  if (NB == 1) return k.b0;
  const uint64_t m0 = (uint64_t)(int64_t)(int32_t)(0u - (e & 1u));          // all ones when bit 0 of e is set
  const uint64_t lo = k.b0 ^ ((k.b0 ^ k.b1) & m0);
  if (NB == 2) return lo;
  const uint64_t hi = k.b2 ^ ((k.b2 ^ k.b3) & m0);
  const uint64_t m1 = (uint64_t)(int64_t)(int32_t)(0u - ((e >> 1) & 1u));   // bit 1 of e
  return lo ^ ((lo ^ hi) & m1);
}

// Sparse evaluate of a fired location whose list is entries[lo, hi); `first`
// is this lane's entry lo + lane, already loaded (kNoEntry past the end).
template <int NB>
__device__ __forceinline__ void evaluate_sparse(const DevModel& m, uint64_t* slab, uint32_t lo, uint32_t hi,
                                                uint32_t first, const Masks& k, uint32_t lane) {
  if (first != kNoEntry) {
    const uint64_t s = select_mask<NB>(first, k);
    if (NB == 1 || s) atomicXor((unsigned long long*)&row_of(slab, first), (unsigned long long)s);
  }
  const guint32_p entries = (guint32_p)m.entries;
  for (uint32_t i = lo + 64u + lane; i < hi; i += 64) {
    const uint32_t e = entries[i];
    const uint64_t s = select_mask<NB>(e, k);
    if (NB == 1 || s) atomicXor((unsigned long long*)&row_of(slab, e), (unsigned long long)s);
  }
}

__device__ __forceinline__ void evaluate_dense(const DevModel& m, uint64_t* slab, uint32_t meta, const Masks& k,
                                               uint32_t lane) {
  const uint32_t var0 = meta >> 8;
  if (k.b0) xor_dense(m, slab, var0, k.b0, lane);
  if (k.b1) xor_dense(m, slab, var0 + 1, k.b1, lane);
  if (k.b2) xor_dense(m, slab, var0 + 2, k.b2, lane);
  if (k.b3) xor_dense(m, slab, var0 + 3, k.b3, lane);
}

// Orders the LDS accesses of one wave's lanes around an exchange through
// LDS (no instruction: the wave's LDS operations already run in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS byte address of a shared-memory pointer, and a 64-bit XOR at an LDS
// byte address.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}
__device__ __forceinline__ void lds_xor(uint32_t addr, uint64_t v) {
  __atomic_fetch_xor((__attribute__((address_space(3))) uint64_t*)(uintptr_t)addr, v, __ATOMIC_RELAXED);
}

// Walks bentries[lo, hi) for one shot: each entry is the byte offset
// (row << 3) of a slab row to flip, so each is one XOR of the shot's bit
// (`bit`) into the slab at LDS address `base`.  Eight entry loads are kept
// in flight, and the last 1..7 entries are loaded together as well: the
// table has 8 entries of slack after its end, so the loads that run past the
// list stay inside it (their values are not used).  BASE0: the slab starts
// at LDS address 0, so an entry is its row's address.
template <bool BASE0>
__device__ __forceinline__ void walk_rows(const DevModel& m, uint32_t base, uint32_t lo, uint32_t hi, uint64_t bit) {
  // 32-bit byte offsets from a uniform base, constant steps as immediates
  const SP_GLOBAL_AS char* ce = (const SP_GLOBAL_AS char*)m.bentries;
  if (BASE0) base = 0;
  uint32_t o = lo << 2;
  const uint32_t o1 = hi << 2;
  for (; o + 32 <= o1; o += 32) {
    const SP_GLOBAL_AS uint32_t* pe = (const SP_GLOBAL_AS uint32_t*)(ce + o);
    uint32_t e[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) e[k] = pe[k];
#pragma unroll
    for (int k = 0; k < 8; ++k) lds_xor(base + e[k], bit);
  }
  if (o < o1) {   // the last 1..7 entries: seven loads at once, r XORs
    const SP_GLOBAL_AS uint32_t* pe = (const SP_GLOBAL_AS uint32_t*)(ce + o);
    const uint32_t r = (o1 - o) >> 2;
    uint32_t e[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) e[k] = pe[k];
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if ((uint32_t)k < r) lds_xor(base + e[k], bit);
  }
}

// A wave's record queue (sparse path): record i is the four draws of one
// lane in one block and word, w[i], w[C + i], w[2C + i], w[3C + i] (C =
// kQueueCap), and its tag w[4C + i] = block << 8 | lane << 2 | word, so that a
// lane writes or reads a record at one address and constant offsets.  A lane
// appends a record when any location of the block fired in its shot; the
// four draws say which ones did (u <= T_m - 1, with T_m from the block's hot
// record).
struct Queue {
  uint32_t* w;
};

// Evaluates the queued records, one per lane: the lane reloads its block's
// thresholds, channels and bit-list bounds, and for every location that
// fired in its shot finds the Pauli code from the draw (lane_code) and flips
// its shot's bit in the rows of the code's set bits' columns.  A lane with
// several fired locations takes them one after another.  Everything but the
// queueing is shared by up to 64 records.
template <int R>
__device__ __forceinline__ void flush_records(const DevModel& m, uint64_t* slab, const Queue& q, uint32_t qn,
                                              uint32_t lane) {
  wave_sync();
  if (lane < qn) {
    constexpr uint32_t C = sp::kQueueCap;
    const uint4 u = make_uint4(q.w[lane], q.w[C + lane], q.w[2 * C + lane], q.w[3 * C + lane]);
    const uint32_t tag = q.w[4 * C + lane];
    const uint32_t b = tag >> 8;
    const uint4 tm1 = *(const SP_GLOBAL_AS uint4*)((const SP_GLOBAL_AS char*)m.hot + (b << 5));
    const SP_GLOBAL_AS char* cw = (const SP_GLOBAL_AS char*)m.cold + (b << 6);   // meta | lst | end | btab
    const uint4 meta = *(const SP_GLOBAL_AS uint4*)cw, bt = *(const SP_GLOBAL_AS uint4*)(cw + 48);
    uint32_t fired = (uint32_t)(u.x <= tm1.x) | (uint32_t)(u.y <= tm1.y) << 1 | (uint32_t)(u.z <= tm1.z) << 2 |
                     (uint32_t)(u.w <= tm1.w) << 3;
    const uint64_t bit = 1ull << ((tag >> 2) & 63u);
    const uint32_t base = lds_addr(R == 1 ? slab : slab + (size_t)(tag & 3u) * m.n_meas);
    while (fired) {
      const uint32_t s = (uint32_t)__builtin_ctz(fired);
      fired &= fired - 1u;
      const uint32_t us = s == 0 ? u.x : s == 1 ? u.y : s == 2 ? u.z : u.w;
      const uint32_t mt = s == 0 ? meta.x : s == 1 ? meta.y : s == 2 ? meta.z : meta.w;
      const uint32_t c0 = s == 0 ? bt.x : s == 1 ? bt.y : s == 2 ? bt.z : bt.w;
      // The Pauli of the code flips the XOR of the columns of its set bits:
      // walking each set bit's column flips every row the right number of
      // times (a row in two of them twice, which cancels).  The bits' lists
      // lie one after another, so a run of consecutive set bits is one
      // range.  A slot without a drawn location (threshold 0, fires at u = 0
      // only) has the coin channel and an empty list.
      uint32_t code = lane_code(m.chans, mt & 0xFFu, us);
      while (code) {
        const uint32_t j = (uint32_t)__builtin_ctz(code);
        const uint32_t n = (uint32_t)__builtin_ctz(~(code >> j));   // length of the run from bit j
        code &= ~(((1u << n) - 1u) << j);
        const uint32_t lo = ld32(m.btab, c0 + j), hi = ld32(m.btab, c0 + j + n);
        if (base == 0) walk_rows<true>(m, base, lo, hi, bit);
        else walk_rows<false>(m, base, lo, hi, bit);
      }
    }
  }
  wave_sync();
}

// A block's descriptor: the part every block needs (thresholds, the Philox
// block index and flags, 32 bytes) and the part only evaluated blocks need
// (channels, variables and list bounds, 64 bytes).
struct Hot {
  uint4 tm1;    // T_m - 1 per slot; 0 for a slot without a drawn location
  uint4 blk;    // .x = l / 4; .y bit 0: every drawn slot's channel has a single code
};
struct Cold {
  uint4 meta;   // var0 << 8 | channel + 1 per slot (1 and an empty list: no drawn location)
  uint4 lst;    // start of each slot's entry list
  uint4 end;    // .x = end of slot 3's list
  uint4 btab;   // per slot, where its bit lists' bounds start in btab
};

// The R words of group g: lane t of word r stands for shot
// first_shot + 64 (g R + r) + t.  UHI: every lane's shot index has the same
// high word (the usual case), which lets the first rounds of each draw run
// on the scalar unit.
template <int R, bool UHI>
__device__ __forceinline__ void shot_words(const LaunchArgs& a, uint32_t g, uint32_t lane, const RoundKeys& k,
                                           ShotWord (&w)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) w[r] = shot_word<UHI>(a.first_shot + (uint64_t)(g * R + r) * 64u, lane, k);
}

// Evaluates an eager block whose drawn slots all have single-code channels
// (random measurements, X, Y or Z flips): the mask of each of its variables
// is its slot's fire mask, so the four consecutive entry lists are walked in
// one pass, one entry per lane, each taking its slot's mask.
template <int R>
__device__ __forceinline__ void evaluate_single(const DevModel& m, uint64_t* slab, const Cold* cold, uint32_t b,
                                                const uint64_t (&f)[R][4], uint32_t lane) {
  const Cold c = load_uniform(cold + b);
  const uint32_t lo = c.lst.x, n = c.end.x - lo;
  const uint32_t e1 = c.lst.y - lo, e2 = c.lst.z - lo, e3 = c.lst.w - lo;   // where slots 1..3 start
  const guint32_p entries = (guint32_p)m.entries;
  for (uint32_t i = lane; i < n; i += 64) {
    const uint32_t e = entries[lo + i];
    // All ones from slot k's first entry on (e1 <= e2 <= e3), so that the
    // slot's mask is a telescoping XOR (written as masked XORs, the masks
    // stay scalar operands and no lookup table is formed).
    const uint64_t s1 = (uint64_t)(int64_t)(int32_t)(0u - (uint32_t)(i >= e1));
    const uint64_t s2 = (uint64_t)(int64_t)(int32_t)(0u - (uint32_t)(i >= e2));
    const uint64_t s3 = (uint64_t)(int64_t)(int32_t)(0u - (uint32_t)(i >= e3));
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t mk = f[r][0] ^ ((f[r][0] ^ f[r][1]) & s1) ^ ((f[r][1] ^ f[r][2]) & s2) ^ ((f[r][2] ^ f[r][3]) & s3);
      if (mk) atomicXor((unsigned long long*)&row_of(slab + (size_t)r * m.n_meas, e), (unsigned long long)mk);
    }
  }
}

// Evaluates every fired location of block b now (lane = entry of the
// location's list): eager blocks, whose locations fire in many
// lanes, and every fired block on the dense path.
template <int R, int DENSE>
__device__ __forceinline__ void evaluate_block(const DevModel& m, uint64_t* slab, const Cold* cold, uint32_t b,
                                               const uint4 (&u)[R], const uint64_t (&f)[R][4], uint32_t lane) {
  const Cold c = load_uniform(cold + b);
  const uint4 d1 = c.meta, d2 = c.lst, d3 = c.end;
  // Issue the first entry load of every fired location before decoding, so
  // that their latencies overlap.
  uint32_t first[4] = {kNoEntry, kNoEntry, kNoEntry, kNoEntry};
  if (!DENSE) {
    const guint32_p entries = (guint32_p)m.entries;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      uint64_t any_s = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) any_s |= f[r][s];
      const uint32_t lo = pick(d2, s), hi = s < 3 ? pick(d2, s + 1) : d3.x;
      if (any_s && lo + lane < hi) first[s] = entries[lo + lane];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (!f[r][s]) continue;
      const uint32_t meta = pick(d1, s);
      const uint32_t lo = pick(d2, s), hi = s < 3 ? pick(d2, s + 1) : d3.x;
      if (lo == hi) continue;   // no output depends on it (or no drawn location)
      const Masks k = decode(m.chans, meta, pick(u[r], s), f[r][s], lane);
      uint64_t* sl = slab + (size_t)r * m.n_meas;
      if (DENSE) {
        evaluate_dense(m, sl, meta, k, lane);
      } else {
        if (k.nbits == 1) evaluate_sparse<1>(m, sl, lo, hi, first[s], k, lane);
        else if (k.nbits == 2) evaluate_sparse<2>(m, sl, lo, hi, first[s], k, lane);
        else evaluate_sparse<4>(m, sl, lo, hi, first[s], k, lane);
      }
    }
  }
}

// One block of the draw loop: draw, fire test, then either queue the fired
// lanes' records (QUEUE: the sparse path's lazy blocks) or evaluate every
// fired location at once (eager blocks, and every block on the dense path).
// Returns the hot record at `next`, whose load is issued once the current
// record has been used (scalar loads complete out of order, so a wait for
// the current record would otherwise also wait for the next one).
template <int R, int DENSE, bool QUEUE, bool UHI>
__device__ __forceinline__ Hot draw_block(const LaunchArgs& a, uint64_t* slab, const Queue& q, uint32_t& qn,
                                          const Hot& cur, const Hot* next, uint32_t b, const RoundKeys& keys,
                                          const ShotWord (&w)[R], uint32_t lane4) {
  const DevModel& m = a.m;
  uint4 u[R];
#pragma unroll
  for (int r = 0; r < R; ++r) u[r] = draw4<UHI>(cur.blk.x, w[r], keys);
  // Every word of `cur` is in registers here; keep the next load below.
  asm volatile("" ::"s"(cur.tm1.x), "s"(cur.tm1.y), "s"(cur.tm1.z), "s"(cur.tm1.w) : "memory");
  const Hot nx = load_uniform(next);
  // A slot without a drawn location has threshold 0: it "fires" only at
  // u = 0, and its empty list makes that a no-op.
  bool c[R][4];
  uint64_t f[R][4], fr[R];
  uint64_t any = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    c[r][0] = u[r].x <= cur.tm1.x;
    c[r][1] = u[r].y <= cur.tm1.y;
    c[r][2] = u[r].z <= cur.tm1.z;
    c[r][3] = u[r].w <= cur.tm1.w;
#pragma unroll
    for (int s = 0; s < 4; ++s) f[r][s] = ballot(c[r][s]);
    fr[r] = f[r][0] | f[r][1] | f[r][2] | f[r][3];
    any |= fr[r];
  }
  if (!any) return nx;   // the usual case at p ~ 1e-3: nothing fired in this block
  if (!QUEUE) {
    if (!DENSE && (cur.blk.y & 1u)) evaluate_single<R>(m, slab, reinterpret_cast<const Cold*>(m.cold), b, f, lane4 >> 2);
    else evaluate_block<R, DENSE>(m, slab, reinterpret_cast<const Cold*>(m.cold), b, u, f, lane4 >> 2);
    return nx;
  }
  // Queue one record per fired lane and word.  A word's records always fit
  // an emptied queue: it has at most 64 fired lanes.
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (R > 1 && !fr[r]) continue;
    const uint32_t n = (uint32_t)__builtin_popcountll(fr[r]);
    if (qn + n > sp::kQueueCap) {
      flush_records<R>(m, slab, q, qn, lane4 >> 2);
      qn = 0;
    }
    constexpr uint32_t C = sp::kQueueCap;
    uint32_t* qd = q.w + qn;   // wave-uniform base
    const uint32_t tag = (b << 8) | (uint32_t)r;
    if (c[r][0] | c[r][1] | c[r][2] | c[r][3]) {   // this lane's shot fired somewhere in the block
      const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(fr[r] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fr[r], 0u));
      qd[pos] = u[r].x;
      qd[C + pos] = u[r].y;
      qd[2 * C + pos] = u[r].z;
      qd[3 * C + pos] = u[r].w;
      qd[4 * C + pos] = tag | lane4;
    }
    qn += n;
  }
  return nx;
}

// The blocks [b0, b1) of the hot table that one wave draws: b0 + wave,
// b0 + wave + n_waves, ...  Two blocks per iteration, so that the record
// loaded one block ahead lands in the registers of the block after next and
// no record is copied; the hot table's padding makes the load past the last
// block safe.
template <int R, int DENSE, bool QUEUE, bool UHI>
__device__ __forceinline__ void draw_range(const LaunchArgs& a, uint64_t* slab, const Queue& q, uint32_t& qn,
                                           uint32_t b0, uint32_t b1, const RoundKeys& keys, const ShotWord (&w)[R],
                                           uint32_t wave, uint32_t n_waves, uint32_t lane4) {
  uint32_t b = b0 + wave;
  if (b >= b1) return;
  const Hot* hot = reinterpret_cast<const Hot*>(a.m.hot);
  Hot h0 = load_uniform(hot + b);
  for (;;) {
    const Hot h1 = draw_block<R, DENSE, QUEUE, UHI>(a, slab, q, qn, h0, hot + b + n_waves, b, keys, w, lane4);
    b += n_waves;
    if (b >= b1) break;
    h0 = draw_block<R, DENSE, QUEUE, UHI>(a, slab, q, qn, h1, hot + b + n_waves, b, keys, w, lane4);
    b += n_waves;
    if (b >= b1) break;
  }
}

// The draw-select-evaluate loop of one wave over its share of the blocks:
// the lazy blocks [0, nb_lazy) queue their fired lanes (sparse path), the
// eager ones [nb_lazy, nb) are evaluated at once; on the dense path every
// block is evaluated at once.
template <int R, int DENSE, bool UHI>
__device__ __forceinline__ void run_blocks(const LaunchArgs& a, uint64_t* slab, const Queue& q, uint32_t g,
                                           uint32_t wave, uint32_t n_waves, uint32_t lane) {
  const DevModel& m = a.m;
  if (wave >= m.nb) return;
  RoundKeys keys = round_keys(a.key0, a.key1);
  // Rounds 4..9 run on the vector unit alone: their keys in VGPRs (a copy in
  // every lane) leave the scalar registers to the rest, so that eight waves
  // per SIMD fit.
#pragma unroll
  for (int r = 4; r < 10; ++r) {
    keys.k0[r] = to_vgpr(keys.k0[r]);
    keys.k1[r] = to_vgpr(keys.k1[r]);
  }
  ShotWord w[R];
  shot_words<R, UHI>(a, g, lane, keys, w);
  const uint32_t lane4 = lane << 2;
  uint32_t qn = 0;   // queued records (wave-uniform)
  if (DENSE) {
    draw_range<R, DENSE, false, UHI>(a, slab, q, qn, 0, m.nb, keys, w, wave, n_waves, lane4);
    return;
  }
  draw_range<R, DENSE, true, UHI>(a, slab, q, qn, 0, m.nb_lazy, keys, w, wave, n_waves, lane4);
  if (qn) flush_records<R>(m, slab, q, qn, lane);
  draw_range<R, DENSE, false, UHI>(a, slab, q, qn, m.nb_lazy, m.nb, keys, w, wave, n_waves, lane4);
}

// blockIdx -> group, keeping consecutive groups on one XCD (workgroups are
// dealt round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ uint32_t xcd_group(uint32_t b, uint32_t n) {
  const uint32_t q = n / 8u, r = n % 8u;
  const uint32_t x = b % 8u, i = b / 8u;
  return x * q + min(x, r) + i;
}

// One group = R consecutive 64-shot words of one job, each with its LDS
// slab of n_meas rows: initialise from c, draw and evaluate, store.
template <int R, int DENSE>
__device__ __forceinline__ void process_group(const LaunchArgs& a, uint64_t* slab, uint32_t g, uint32_t tid,
                                              uint32_t lane, uint32_t wave, uint32_t n_waves) {
  const DevModel& m = a.m;
  const guint64_p c_mask = (guint64_p)m.c_mask;
  for (uint32_t k = tid; k < m.n_meas; k += blockDim.x) {
    const uint64_t v = ((c_mask[k >> 6] >> (k & 63u)) & 1ull) ? ~0ull : 0ull;
#pragma unroll
    for (int r = 0; r < R; ++r) slab[(size_t)r * m.n_meas + k] = v;
  }
  __syncthreads();

  // Do the R words' shot indices share one high word?
  const uint64_t first = a.first_shot + (uint64_t)g * R * 64u;
  const uint64_t last = first + (uint64_t)R * 64u - 1u;
  // The waves' record queues follow the slabs (16-byte aligned): per wave,
  // kQueueCap records of five words.
  char* qbase = reinterpret_cast<char*>(slab + (((size_t)R * m.n_meas + 1u) & ~(size_t)1)) +
                (size_t)wave * sp::kQueueCap * sp::kQueueRecBytes;
  const Queue queue{reinterpret_cast<uint32_t*>(qbase)};
  if ((first >> 32) == (last >> 32)) run_blocks<R, DENSE, true>(a, slab, queue, g, wave, n_waves, lane);
  else run_blocks<R, DENSE, false>(a, slab, queue, g, wave, n_waves, lane);
  __syncthreads();

#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t w = g * R + r;
    if (w >= a.n_words) break;
    const uint64_t rem = a.shots - (uint64_t)w * 64u;
    const uint64_t valid = rem >= 64u ? ~0ull : ((1ull << rem) - 1ull);
    const gout_p col = (gout_p)a.out + w;
    for (uint32_t k = tid; k < m.n_meas; k += blockDim.x) col[(size_t)k * a.ld] = slab[(size_t)r * m.n_meas + k] & valid;
  }
}

// With one word per group the single-job kernels ask for eight waves per
// SIMD (at most 64 VGPRs and 96 SGPRs): a CU then holds four 8-wave
// workgroups where their LDS fits, which hides the record flush's load
// latency far better than three.  With more words per group the slabs' LDS
// limits the waves anyway, and the limit would spill vector registers; the
// batched kernels, which keep a job's pointers in scalar registers, keep
// the compiler's default too (under the limit those spill, and served
// batches ran 5% slower).
// One job per launch: workgroup b owns group xcd_group(b).
template <int R, int DENSE>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(R == 1 ? 8 : 1))) sample_kernel(LaunchArgs a) {
  extern __shared__ uint64_t slab[];
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = uniform(tid >> 6), n_waves = blockDim.x >> 6;
  process_group<R, DENSE>(a, slab, xcd_group(blockIdx.x, a.n_groups), tid, lane, wave, n_waves);
}

// Every row tile of one model in one launch.  The flat index group * n_tiles
// + tile is spread over the XCDs like a single tile's groups, so each XCD
// takes a run of consecutive words of every tile and all tiles advance
// together (tiles of unequal cost then share every XCD); each workgroup
// reads its tile's record from the table with scalar loads.
template <int R, int DENSE>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(R == 1 ? 8 : 1))) sample_tiles_kernel(TiledArgs t) {
  extern __shared__ uint64_t slab[];
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = uniform(tid >> 6), n_waves = blockDim.x >> 6;
  const uint32_t f = xcd_group(blockIdx.x, t.n_tiles * t.n_groups);
  const uint32_t ti = f % t.n_tiles;
  const TileRec rec = load_uniform(t.tiles + ti);
  LaunchArgs a;
  a.m = rec.m;
  a.out = t.out + (size_t)rec.row0 * t.ld;
  a.ld = t.ld;
  a.first_shot = t.first_shot;
  a.shots = t.shots;
  a.key0 = t.key0;
  a.key1 = t.key1;
  a.n_words = t.n_words;
  a.n_groups = t.n_groups;
  process_group<R, DENSE>(a, slab, f / t.n_tiles, tid, lane, wave, n_waves);
}

// Group g of a batched job: the tile's model and output rows for a job over
// row tiles, else the job itself.
template <int R, int DENSE>
__device__ __forceinline__ void process_job_group(const BatchJob& job, uint64_t* slab, uint32_t g, uint32_t tid,
                                                  uint32_t lane, uint32_t wave, uint32_t n_waves) {
  LaunchArgs a = job.a;
  if (job.n_tiles > 1) {
    const uint32_t ti = g % job.n_tiles;
    const TileRec rec = load_uniform(job.tiles + ti);
    a.m = rec.m;
    a.out = job.a.out + (size_t)rec.row0 * job.a.ld;
    g /= job.n_tiles;
  }
  process_group<R, DENSE>(a, slab, g, tid, lane, wave, n_waves);
}

// Many jobs per launch, persistent schedule: workgroups take tasks (runs of
// consecutive groups of one job) from a device counter until all are handed
// out.  The workgroup that finishes last resets the counters, so the launch
// can be replayed (for example from a captured graph) without any host-side
// reset.
template <int R, int DENSE>
__global__ void __launch_bounds__(1024) batch_persistent_kernel(const BatchJob* __restrict__ jobs,
                                                                const sp::BatchTask* __restrict__ tasks,
                                                                uint32_t n_tasks, BatchCounters* ctr) {
  extern __shared__ uint64_t slab[];
  __shared__ uint32_t s_next;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = uniform(tid >> 6), n_waves = blockDim.x >> 6;
  if (tid == 0) s_next = atomicAdd(&ctr->next, 1u);
  __syncthreads();
  uint32_t t = uniform(s_next);
  while (t < n_tasks) {
    uint32_t nxt = 0;
    if (tid == 0) nxt = atomicAdd(&ctr->next, 1u);   // next task, in flight during this one
    const sp::BatchTask task = load_uniform(tasks + t);
    const BatchJob job = load_uniform(jobs + task.job);
    for (uint32_t i = 0; i < task.count; ++i) {
      process_job_group<R, DENSE>(job, slab, task.first + i, tid, lane, wave, n_waves);
      __syncthreads();
    }
    if (tid == 0) s_next = nxt;
    __syncthreads();
    t = uniform(s_next);
  }
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(&ctr->done, 1u) == gridDim.x - 1u) {
      atomicExch(&ctr->next, 0u);
      atomicExch(&ctr->done, 0u);
      __threadfence();
    }
  }
}

// blockIdx -> group within runs of 64: the dispatcher deals workgroups
// round-robin over the 8 XCDs, so XCD x receives groups 8x .. 8x+7 of each
// run (consecutive words of a job, adjacent in every output row); the runs
// themselves keep their order.  The last partial run maps to itself.
__device__ __forceinline__ uint32_t run_swizzle(uint32_t b, uint32_t n) {
  if ((b | 63u) >= n) return b;
  return (b & ~63u) | ((b & 7u) << 3) | ((b >> 3) & 7u);
}

// Many jobs per launch, flat schedule: one workgroup per group (jobs are
// ordered heaviest first, so the hardware dispatcher hands out the
// expensive groups first).
template <int R, int DENSE>
__global__ void __launch_bounds__(1024) batch_flat_kernel(const BatchJob* __restrict__ jobs,
                                                          const uint32_t* __restrict__ group_job, uint32_t total) {
  extern __shared__ uint64_t slab[];
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = uniform(tid >> 6), n_waves = blockDim.x >> 6;
  const uint32_t g = run_swizzle(blockIdx.x, total);
  const BatchJob job = load_uniform(jobs + ((cuint32_p)group_job)[g]);
  process_job_group<R, DENSE>(job, slab, g - job.group_base, tid, lane, wave, n_waves);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Locations that fire in at least an eighth of the shots (T_m >= 2^29) make
// their block eager: evaluated at once, lane = list entry, which costs less
// than queueing their many fired lanes one record each.
constexpr uint64_t kEagerTm = 1ull << 29;

// Drawn locations grouped by Philox block (l/4); blocks without a drawn
// location are left out.  The lazy blocks come first, then the eager ones
// (nb_lazy counts the former), each part in block order; the order of blocks
// changes no output, since every draw is keyed by its block index.  Per
// block, a hot record of 8 words:
//   [0..3]  T_m - 1 per slot (fire when u <= T_m - 1, i.e. u < T_m); 0 for
//           a slot without a drawn location
//   [4]     the Philox block index l/4
//   [5]     1 when every drawn slot's channel has a single code (its
//           variable's mask is the fire mask), else 0
// followed, after the last block, by kHotPad zero records (read, never used),
// and a cold record of 16 words:
//   [0..3]  meta per slot: var0 << 8 | (channel + 1); 1 (channel 0, with an
//           empty list) for a slot without a drawn location
//   [4..7]  start of the slot's entry list; [8] end of slot 3's list
//   [12..15] per slot, the start of its bit-list bounds in btab (0 for a
//           slot without a drawn location: the empty range [0, 0])
// Entry lists: for every variable of the location (bit b), for every row k
// of its column of M, the word k << 5 | b (so that e >> 2 is the row's LDS
// byte offset and bits 0..4 of e are the bit index).
// Bit lists: the same columns without the bit tags, each row as its byte
// offset k << 3, bit after bit; btab holds a location's nbits + 1 bounds.
struct HostBlocks {
  std::vector<uint32_t> hot, cold;
  std::vector<uint32_t> entries;
  std::vector<uint32_t> btab, bentries;
  uint32_t nb_lazy = 0;
};

// Output rows [r0, r1) only (a row tile): a location is kept when some row of
// the range depends on it, and its entries name rows relative to r0.
bool loc_reaches(const sp_model& m, uint32_t l, uint32_t r0, uint32_t r1) {
  const uint32_t v0 = (uint32_t)m.loc_var0[l];
  for (uint32_t b = 0; b < sp::loc_bits(m.loc_kind[l]); ++b) {
    const uint32_t* lo = m.row_idx.data() + m.col_ptr[v0 + b];
    const uint32_t* hi = m.row_idx.data() + m.col_ptr[v0 + b + 1];
    const uint32_t* it = std::lower_bound(lo, hi, r0);   // rows ascend within a column
    if (it != hi && *it < r1) return true;
  }
  return false;
}

HostBlocks build_blocks(const sp_model& m, uint32_t r0, uint32_t r1) {
  HostBlocks H;
  if (m.n_meas >= (1u << 27)) throw sp::Error(SP_E_LIMIT, "more than 2^27 measurements");
  if (m.n_locs >= (1u << 24)) throw sp::Error(SP_E_LIMIT, "more than 2^24 locations");
  const bool whole = r0 == 0 && r1 >= m.n_meas;
  int64_t cur = -1;
  std::vector<uint8_t> eager;   // per block
  H.btab = {0u, 0u};            // the empty range of slots without a drawn location
  std::vector<uint32_t> rows[4];
  for (uint32_t l = 0; l < m.n_locs; ++l) {
    if (!sp::loc_drawn(m, l)) continue;   // never fires, or reaches no output row
    if (!whole && !loc_reaches(m, l, r0, r1)) continue;
    const int32_t ch = m.loc_chan[l];
    const sp::Channel& c = m.channels[ch];
    const uint64_t Tm = c.T[c.m];
    const int64_t blk = l >> 2;
    if (blk != cur) {
      H.hot.insert(H.hot.end(), 8, 0u);
      H.cold.insert(H.cold.end(), 16, 0u);
      uint32_t* w = &H.cold[H.cold.size() - 16];
      for (int i = 0; i < 4; ++i) w[i] = 1u;   // empty slot: the coin channel, empty list
      for (int i = 4; i <= 8; ++i) w[i] = (uint32_t)H.entries.size();
      H.hot[H.hot.size() - 8 + 4] = (uint32_t)blk;
      H.hot[H.hot.size() - 8 + 5] = 1u;   // every drawn slot single-code, until one is not
      eager.push_back(0);
      cur = blk;
    }
    uint32_t* h = &H.hot[H.hot.size() - 8];
    uint32_t* w = &H.cold[H.cold.size() - 16];
    const uint32_t s = l & 3u, var0 = (uint32_t)m.loc_var0[l];
    h[s] = (uint32_t)(Tm - 1);
    if (c.m != 1) h[5] = 0u;
    if (Tm >= kEagerTm) eager.back() = 1;
    w[s] = (var0 << 8) | (uint32_t)(ch + 1);
    w[4 + s] = (uint32_t)H.entries.size();
    const uint32_t nbits = sp::loc_bits(m.loc_kind[l]);
    for (uint32_t b = 0; b < nbits; ++b) {
      rows[b].clear();
      for (uint32_t i = m.col_ptr[var0 + b]; i < m.col_ptr[var0 + b + 1]; ++i) {
        const uint32_t k = m.row_idx[i];
        if (k >= r0 && k < r1) {
          H.entries.push_back(((k - r0) << 5) | b);
          rows[b].push_back(k - r0);
        }
      }
    }
    w[12 + s] = (uint32_t)H.btab.size();
    H.btab.push_back((uint32_t)H.bentries.size());
    for (uint32_t b = 0; b < nbits; ++b) {
      for (uint32_t k : rows[b]) H.bentries.push_back(k << 3);
      H.btab.push_back((uint32_t)H.bentries.size());
    }
    if (H.entries.size() >= (1ull << 32)) throw sp::Error(SP_E_LIMIT, "more than 2^32 entries in M");
    if (H.bentries.size() >= (1ull << 30) || H.btab.size() >= (1ull << 30))
      throw sp::Error(SP_E_LIMIT, "more than 2^30 bit-list entries (kernels address them with 32-bit offsets)");
    for (uint32_t t = s + 1; t <= 4; ++t) w[4 + t] = (uint32_t)H.entries.size();
  }
  // Lazy blocks first, then eager ones, each part keeping its order.
  std::vector<uint32_t> hot, cold;
  hot.reserve(H.hot.size());
  cold.reserve(H.cold.size());
  for (int pass = 0; pass < 2; ++pass)
    for (size_t i = 0; i < eager.size(); ++i) {
      if (eager[i] != pass) continue;
      hot.insert(hot.end(), H.hot.begin() + 8 * i, H.hot.begin() + 8 * (i + 1));
      cold.insert(cold.end(), H.cold.begin() + 16 * i, H.cold.begin() + 16 * (i + 1));
      if (pass == 0) ++H.nb_lazy;
    }
  H.hot.swap(hot);
  H.cold.swap(cold);
  return H;
}

int choose_path(const sp_model& m, int path) {
  if (path != SP_PATH_AUTO) return path;
  // Dense costs ceil(n_meas/64) LDS operations per fired variable, sparse
  // ceil(|location list|/64): pick dense only when columns are long compared
  // with the slab.
  const double avg = m.n_vars ? (double)m.row_idx.size() / m.n_vars : 0.0;
  return (avg * 4.0 > (double)m.n_meas) ? SP_PATH_DENSE : SP_PATH_SPARSE;
}

// Rows of one LDS slab that leave room for the record queues of 16 waves
// (160 KB of LDS per workgroup on gfx950): the largest tile.  The automatic
// choice keeps one tile while two 8-wave workgroups' slabs and queues fit a
// CU (8,960 rows); past that, a single slab leaves too few waves per SIMD to
// hide the draw's latency, and tiles of 3,840 rows (four workgroups' slabs
// and queues per CU) sample faster despite the draws that several tiles
// repeat.
constexpr uint32_t kSlabRowsMax = (160u * 1024u - 16u * sp::kQueueCap * sp::kQueueRecBytes) / 8u;
constexpr uint32_t kOneTileRowsMax = (80u * 1024u - 8u * sp::kQueueCap * sp::kQueueRecBytes) / 8u;
constexpr uint32_t kTileRowsAuto = 3840;

struct TileLayout {
  size_t hot, cold, entries, btab, bentries, c_mask, dense;
  uint32_t r0, rows, nb, nb_lazy, dense_words;
};

struct Layout {
  std::vector<TileLayout> tiles;
  std::vector<HostBlocks> blocks;
  size_t chans, table, total;   // table: the TileRec array (more than one tile)
  uint32_t nch;
};

static_assert(sizeof(TileRec) % 16 == 0, "tile records are read with 16-byte loads");
static_assert(sizeof(BatchJob) % 16 == 0, "jobs are read with 16-byte loads");

// tile_rows: 0 picks one tile up to kOneTileRowsMax rows, else tiles of
// kTileRowsAuto rows; otherwise tiles of that many rows (a multiple of 64).
Layout plan(const sp_model& m, int path, uint32_t tile_rows) {
  Layout L{};
  uint32_t per = tile_rows;
  if (per == 0) per = m.n_meas <= kOneTileRowsMax ? std::max<uint32_t>(m.n_meas, 1) : kTileRowsAuto;
  L.nch = (uint32_t)m.channels.size();
  size_t off = 0;
  L.chans = off;
  off = align256(off + 64 * (size_t)L.nch);
  for (uint32_t r0 = 0; r0 < std::max<uint32_t>(m.n_meas, 1); r0 += per) {
    const uint32_t r1 = std::min<uint32_t>(std::max<uint32_t>(m.n_meas, 1), r0 + per);
    L.blocks.push_back(build_blocks(m, r0, r1));
    const HostBlocks& H = L.blocks.back();
    TileLayout T{};
    T.r0 = r0;
    T.rows = m.n_meas ? r1 - r0 : 0;
    T.nb = (uint32_t)(H.hot.size() / 8);
    T.nb_lazy = H.nb_lazy;
    T.dense_words = (T.rows + 63) / 64;
    T.hot = off;     off = align256(off + 32 * ((size_t)T.nb + sp::kHotPad));
    T.cold = off;    off = align256(off + 64 * std::max<size_t>(T.nb, 1));
    T.entries = off; off = align256(off + 4 * std::max<size_t>(H.entries.size(), 1));
    T.btab = off;    off = align256(off + 4 * std::max<size_t>(H.btab.size(), 1));
    T.bentries = off; off = align256(off + 4 * (H.bentries.size() + 8));   // + slack read by walk_rows
    T.c_mask = off;  off = align256(off + 8 * std::max<size_t>(T.dense_words, 1));
    T.dense = off;
    if (path == SP_PATH_DENSE) off = align256(off + 8 * (size_t)m.n_vars * (T.dense_words + (T.dense_words + 63) / 64));
    L.tiles.push_back(T);
  }
  L.table = off;
  if (L.tiles.size() > 1) off = align256(off + sizeof(TileRec) * L.tiles.size());
  L.total = off;
  return L;
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return set_error(SP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

using KernelFn = void (*)(LaunchArgs);
using TilesFn = void (*)(TiledArgs);
using PersistentFn = void (*)(const BatchJob*, const sp::BatchTask*, uint32_t, BatchCounters*);
using FlatFn = void (*)(const BatchJob*, const uint32_t*, uint32_t);

KernelFn kernel_for(int path, uint32_t words_per_group) {
  const bool dense = path == SP_PATH_DENSE;
  switch (words_per_group) {
    case 1: return dense ? sample_kernel<1, 1> : sample_kernel<1, 0>;
    case 2: return dense ? sample_kernel<2, 1> : sample_kernel<2, 0>;
    case 4: return dense ? sample_kernel<4, 1> : sample_kernel<4, 0>;
    default: return nullptr;
  }
}

TilesFn tiles_for(int path, uint32_t words_per_group) {
  const bool dense = path == SP_PATH_DENSE;
  switch (words_per_group) {
    case 1: return dense ? sample_tiles_kernel<1, 1> : sample_tiles_kernel<1, 0>;
    case 2: return dense ? sample_tiles_kernel<2, 1> : sample_tiles_kernel<2, 0>;
    case 4: return dense ? sample_tiles_kernel<4, 1> : sample_tiles_kernel<4, 0>;
    default: return nullptr;
  }
}

PersistentFn persistent_for(int path, uint32_t words_per_group) {
  const bool dense = path == SP_PATH_DENSE;
  switch (words_per_group) {
    case 1: return dense ? batch_persistent_kernel<1, 1> : batch_persistent_kernel<1, 0>;
    case 2: return dense ? batch_persistent_kernel<2, 1> : batch_persistent_kernel<2, 0>;
    case 4: return dense ? batch_persistent_kernel<4, 1> : batch_persistent_kernel<4, 0>;
    default: return nullptr;
  }
}

FlatFn flat_for(int path, uint32_t words_per_group) {
  const bool dense = path == SP_PATH_DENSE;
  switch (words_per_group) {
    case 1: return dense ? batch_flat_kernel<1, 1> : batch_flat_kernel<1, 0>;
    case 2: return dense ? batch_flat_kernel<2, 1> : batch_flat_kernel<2, 0>;
    case 4: return dense ? batch_flat_kernel<4, 1> : batch_flat_kernel<4, 0>;
    default: return nullptr;
  }
}

}  // namespace

namespace sp {

size_t lds_bytes(uint32_t n_meas, uint32_t words_per_group, uint32_t waves_per_group, int path) {
  const size_t slabs = ((size_t)n_meas * words_per_group + 1u) / 2u * 16u;
  return path == SP_PATH_DENSE ? slabs : slabs + (size_t)waves_per_group * kQueueCap * kQueueRecBytes;
}

int launch_sample(const LaunchArgs& a, int path, const sp_launch& L, hipStream_t s) {
  const size_t lds = lds_bytes(a.m.n_meas, L.words_per_group, L.waves_per_group, path);
  KernelFn k = kernel_for(path, L.words_per_group);
  if (!k) return set_error(SP_E_INVALID, "words_per_group must be 1, 2 or 4");
  if (lds > 64 * 1024) HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k, dim3(a.n_groups), dim3(64 * L.waves_per_group), lds, s, a);
  HIP_TRY(hipGetLastError());
  return SP_OK;
}

int launch_sample_tiles(const TiledArgs& a, uint32_t rows_max, int path, const sp_launch& L, hipStream_t s) {
  TilesFn k = tiles_for(path, L.words_per_group);
  if (!k) return set_error(SP_E_INVALID, "words_per_group must be 1, 2 or 4");
  const uint64_t grid = (uint64_t)a.n_tiles * a.n_groups;
  if (grid > 0x7FFFFFFFull) return set_error(SP_E_LIMIT, "too many workgroups for one launch");
  const size_t lds = lds_bytes(rows_max, L.words_per_group, L.waves_per_group, path);
  if (lds > 64 * 1024) HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k, dim3((uint32_t)grid), dim3(64 * L.waves_per_group), lds, s, a);
  HIP_TRY(hipGetLastError());
  return SP_OK;
}

int batch_grid(const sp_launch& L, uint32_t n_meas_max, int path, uint32_t* grid) {
  PersistentFn k = persistent_for(path, L.words_per_group);
  if (!k) return set_error(SP_E_INVALID, "words_per_group must be 1, 2 or 4");
  const size_t lds = lds_bytes(n_meas_max, L.words_per_group, L.waves_per_group, path);
  if (lds > 64 * 1024) HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int dev = 0, cus = 0, per_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k, 64 * L.waves_per_group, lds));
  if (per_cu < 1) return set_error(SP_E_LIMIT, "batched kernel does not fit on a CU with this launch shape");
  *grid = (uint32_t)(cus * per_cu);
  return SP_OK;
}

int launch_batch_persistent(const BatchJob* jobs, const BatchTask* tasks, uint32_t n_tasks, BatchCounters* ctr,
                            uint32_t n_meas_max, int path, const sp_launch& L, uint32_t grid, hipStream_t s) {
  PersistentFn k = persistent_for(path, L.words_per_group);
  if (!k) return set_error(SP_E_INVALID, "words_per_group must be 1, 2 or 4");
  const size_t lds = lds_bytes(n_meas_max, L.words_per_group, L.waves_per_group, path);
  if (lds > 64 * 1024) HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * L.waves_per_group), lds, s, jobs, tasks, n_tasks, ctr);
  HIP_TRY(hipGetLastError());
  return SP_OK;
}

int launch_batch_flat(const BatchJob* jobs, const uint32_t* group_job, uint32_t total_groups, uint32_t n_meas_max,
                      int path, const sp_launch& L, hipStream_t s) {
  FlatFn k = flat_for(path, L.words_per_group);
  if (!k) return set_error(SP_E_INVALID, "words_per_group must be 1, 2 or 4");
  const size_t lds = lds_bytes(n_meas_max, L.words_per_group, L.waves_per_group, path);
  if (lds > 64 * 1024) HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k, dim3(total_groups), dim3(64 * L.waves_per_group), lds, s, jobs, group_job, total_groups);
  HIP_TRY(hipGetLastError());
  return SP_OK;
}

}  // namespace sp

namespace {

// Default launch: 8 waves per group; two words per group when three such
// groups fit in the LDS of a CU (more shots per descriptor fetch), else one.
sp_launch default_launch(const sp_dmodel& dm) {
  sp_launch L;
  L.waves_per_group = 8;
  L.words_per_group = (sp::lds_bytes(dm.rows_max, 2, 8, dm.path) * 3 <= dm.lds_max) ? 2 : 1;
  return L;
}

int validate_launch(const sp_dmodel& dm, const sp_launch& L) {
  if (L.waves_per_group < 1 || L.waves_per_group > 16) return set_error(SP_E_INVALID, "waves_per_group must be 1..16");
  if (!kernel_for(dm.path, L.words_per_group)) return set_error(SP_E_INVALID, "words_per_group must be 1, 2 or 4");
  if (sp::lds_bytes(dm.rows_max, L.words_per_group, L.waves_per_group, dm.path) > dm.lds_max)
    return set_error(SP_E_LIMIT, "words_per_group slabs exceed the LDS of one workgroup");
  return SP_OK;
}

int check_tile_rows(uint32_t tile_rows) {
  if (tile_rows % 64 != 0 || tile_rows > kSlabRowsMax)
    return set_error(SP_E_INVALID, "tile_rows must be 0 or a multiple of 64 up to " + std::to_string(kSlabRowsMax));
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_model_device_bytes_tiled(const sp_model* model, int path, uint32_t tile_rows, size_t* bytes) {
  if (!model || !bytes) return set_error(SP_E_INVALID, "null argument");
  if (path < SP_PATH_AUTO || path > SP_PATH_DENSE) return set_error(SP_E_INVALID, "unknown path");
  if (int rc = check_tile_rows(tile_rows)) return rc;
  try {
    *bytes = plan(*model, choose_path(*model, path), tile_rows).total;
  } catch (const sp::Error& e) {
    return set_error(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  return SP_OK;
}

int sp_model_device_bytes(const sp_model* model, int path, size_t* bytes) {
  return sp_model_device_bytes_tiled(model, path, 0, bytes);
}

int sp_model_upload_tiled(const sp_model* model, int path, uint32_t tile_rows, void* d_buf, size_t buf_bytes,
                          void* stream, sp_dmodel** out) {
  if (!model || !d_buf || !out) return set_error(SP_E_INVALID, "null argument");
  *out = nullptr;
  if (path < SP_PATH_AUTO || path > SP_PATH_DENSE) return set_error(SP_E_INVALID, "unknown path");
  if (((uintptr_t)d_buf & 255u) != 0) return set_error(SP_E_INVALID, "device buffer must be 256-byte aligned");
  if (model->channels.size() > 255) return set_error(SP_E_LIMIT, "more than 255 distinct channels");
  if (int rc = check_tile_rows(tile_rows)) return rc;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  int lds_max = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const int p = choose_path(*model, path);
  std::vector<uint8_t> host;
  Layout L;
  uint32_t rows_max = 0;
  try {
    L = plan(*model, p, tile_rows);
    for (const TileLayout& T : L.tiles) rows_max = std::max(rows_max, T.rows);
    if (sp::lds_bytes(rows_max, 1, 1, p) > (size_t)lds_max)
      return set_error(SP_E_LIMIT, "a tile of " + std::to_string(rows_max) + " rows needs " +
                                       std::to_string(sp::lds_bytes(rows_max, 1, 1, p)) +
                                       " bytes of LDS; the device allows " + std::to_string(lds_max));
    if (buf_bytes < L.total)
      return set_error(SP_E_INVALID, "device buffer of " + std::to_string(buf_bytes) + " bytes, need " +
                                         std::to_string(L.total));
    host.assign(L.total, 0);
    for (uint32_t c = 0; c < L.nch; ++c) {
      uint32_t* t = reinterpret_cast<uint32_t*>(&host[L.chans + 64 * (size_t)c]);
      const sp::Channel& ch = model->channels[c];
      t[0] = ch.kind | (ch.m << 8);
      for (uint32_t k = 1; k < 16; ++k) t[k] = k < ch.m ? (uint32_t)ch.T[k] : 0xFFFFFFFFu;
    }
    for (size_t ti = 0; ti < L.tiles.size(); ++ti) {
      const TileLayout& T = L.tiles[ti];
      const HostBlocks& H = L.blocks[ti];
      if (!H.hot.empty()) std::memcpy(&host[T.hot], H.hot.data(), 4 * H.hot.size());
      if (!H.cold.empty()) std::memcpy(&host[T.cold], H.cold.data(), 4 * H.cold.size());
      if (!H.entries.empty()) std::memcpy(&host[T.entries], H.entries.data(), 4 * H.entries.size());
      if (!H.btab.empty()) std::memcpy(&host[T.btab], H.btab.data(), 4 * H.btab.size());
      if (!H.bentries.empty()) std::memcpy(&host[T.bentries], H.bentries.data(), 4 * H.bentries.size());
      // c of rows [r0, r0 + rows), shifted to start at bit 0
      uint64_t* cm = reinterpret_cast<uint64_t*>(&host[T.c_mask]);
      for (uint32_t k = 0; k < T.rows; ++k) {
        const uint32_t g = T.r0 + k;
        if ((model->c_bits[g >> 6] >> (g & 63)) & 1ull) cm[k >> 6] |= 1ull << (k & 63);
      }
      if (p == SP_PATH_DENSE) {
        // Per variable: the bitmap of its non-zero words, then the words.
        uint64_t* d = reinterpret_cast<uint64_t*>(&host[T.dense]);
        const size_t nzw = (T.dense_words + 63) / 64, stride = T.dense_words + nzw;
        for (uint32_t j = 0; j < model->n_vars; ++j)
          for (uint32_t i = model->col_ptr[j]; i < model->col_ptr[j + 1]; ++i) {
            const uint32_t k = model->row_idx[i];
            if (k < T.r0 || k >= T.r0 + T.rows) continue;
            const uint32_t w = (k - T.r0) >> 6;
            d[(size_t)j * stride + nzw + w] |= 1ull << ((k - T.r0) & 63);
            d[(size_t)j * stride + (w >> 6)] |= 1ull << (w & 63);
          }
      }
    }
  } catch (const sp::Error& e) {
    return set_error(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  auto* dm = new (std::nothrow) sp_dmodel();
  if (!dm) return set_error(SP_E_NOMEM, "out of host memory");
  const uint8_t* base = (const uint8_t*)d_buf;
  try {
    for (const TileLayout& T : L.tiles) {
      sp::DevModel m{};
      m.hot = (const uint4*)(base + T.hot);
      m.cold = (const uint4*)(base + T.cold);
      m.entries = (const uint32_t*)(base + T.entries);
      m.btab = (const uint32_t*)(base + T.btab);
      m.bentries = (const uint32_t*)(base + T.bentries);
      m.chans = (const uint32_t*)(base + L.chans);
      m.c_mask = (const uint64_t*)(base + T.c_mask);
      m.dense = p == SP_PATH_DENSE ? (const uint64_t*)(base + T.dense) : nullptr;
      m.nb = T.nb;
      m.nb_lazy = T.nb_lazy;
      m.nch = L.nch;
      m.n_meas = T.rows;
      m.dense_words = T.dense_words;
      dm->tiles.push_back(m);
      dm->row0.push_back(T.r0);
      dm->nb += T.nb;
    }
  } catch (const std::bad_alloc&) {
    delete dm;
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  dm->d_tiles = nullptr;
  if (L.tiles.size() > 1) {
    TileRec* rec = reinterpret_cast<TileRec*>(&host[L.table]);
    for (size_t t = 0; t < L.tiles.size(); ++t) {
      rec[t] = TileRec{};
      rec[t].m = dm->tiles[t];
      rec[t].row0 = dm->row0[t];
    }
    dm->d_tiles = (const TileRec*)(base + L.table);
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(d_buf, host.data(), L.total, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete dm;
    return set_error(SP_E_DEVICE, std::string("model upload: ") + hipGetErrorString(e));
  }
  dm->n_meas = model->n_meas;
  dm->rows_max = rows_max;
  dm->path = p;
  dm->device = dev;
  dm->lds_max = (size_t)lds_max;
  sp_model_dims(model, &dm->dims);
  dm->launch = default_launch(*dm);
  *out = dm;
  return SP_OK;
}

int sp_model_upload(const sp_model* model, int path, void* d_buf, size_t buf_bytes, void* stream, sp_dmodel** out) {
  return sp_model_upload_tiled(model, path, 0, d_buf, buf_bytes, stream, out);
}

void sp_dmodel_free(sp_dmodel* dm) { delete dm; }

int sp_dmodel_dims(const sp_dmodel* dm, sp_dims* out) {
  if (!dm || !out) return set_error(SP_E_INVALID, "null argument");
  *out = dm->dims;
  return SP_OK;
}

int sp_dmodel_tiles(const sp_dmodel* dm, uint32_t* n_tiles, uint32_t* rows_max) {
  if (!dm) return set_error(SP_E_INVALID, "null model");
  if (n_tiles) *n_tiles = (uint32_t)dm->tiles.size();
  if (rows_max) *rows_max = dm->rows_max;
  return SP_OK;
}

int sp_dmodel_get_launch(const sp_dmodel* dm, sp_launch* out) {
  if (!dm || !out) return set_error(SP_E_INVALID, "null argument");
  *out = dm->launch;
  return SP_OK;
}

int sp_dmodel_set_launch(sp_dmodel* dm, const sp_launch* launch) {
  if (!dm) return set_error(SP_E_INVALID, "null model");
  const sp_launch L = launch ? *launch : default_launch(*dm);
  int rc = validate_launch(*dm, L);
  if (rc) return rc;
  dm->launch = L;
  return SP_OK;
}

int sp_sample(const sp_dmodel* dm, uint64_t seed, uint64_t first_shot, uint64_t shots, uint64_t* d_out,
              size_t ld_words, void* stream) {
  if (!dm) return set_error(SP_E_INVALID, "null model");
  if (shots == 0 || dm->n_meas == 0) return SP_OK;
  if (!d_out) return set_error(SP_E_INVALID, "null output");
  if (((uintptr_t)d_out & 7u) != 0) return set_error(SP_E_INVALID, "output must be 8-byte aligned");
  const uint64_t words = (shots + 63) / 64;
  if (ld_words < words) return set_error(SP_E_INVALID, "ld_words " + std::to_string(ld_words) + " < " + std::to_string(words));
  if (words > 0x7FFFFFFFull) return set_error(SP_E_LIMIT, "too many shots for one launch");
  if (first_shot + shots < first_shot) return set_error(SP_E_INVALID, "shot range overflows 64 bits");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != dm->device) return set_error(SP_E_INVALID, "current device differs from the model's device");
  const sp_launch& L = dm->launch;

  const uint32_t n_groups = (uint32_t)((words + L.words_per_group - 1) / L.words_per_group);
  if (dm->tiles.size() == 1) {
    LaunchArgs a;
    a.m = dm->tiles[0];
    a.out = d_out;
    a.ld = ld_words;
    a.first_shot = first_shot;
    a.shots = shots;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.n_words = (uint32_t)words;
    a.n_groups = n_groups;
    return sp::launch_sample(a, dm->path, L, (hipStream_t)stream);
  }
  // Row tiles: one launch, each tile writing its own rows of the output.
  TiledArgs a;
  a.tiles = dm->d_tiles;
  a.out = d_out;
  a.ld = ld_words;
  a.first_shot = first_shot;
  a.shots = shots;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.n_words = (uint32_t)words;
  a.n_groups = n_groups;
  a.n_tiles = (uint32_t)dm->tiles.size();
  return sp::launch_sample_tiles(a, dm->rows_max, dm->path, L, (hipStream_t)stream);
}

}  // extern "C"

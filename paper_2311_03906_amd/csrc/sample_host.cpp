// Sampling of Algorithm 1 on the host CPU: M_samples = M [b_1 ... b_nsmp] + c
// over GF(2) (Section 3.2.3, Eq. 4), with the same keyed draws and the same
// packed output layout as the GPU kernels (sp_sample).
//
// This is the paper's own method on a CPU (its Section 5 evaluates the
// product with sparse column lists), written for 64 shots at a time: a
// thread owns a run of 64-shot words; for each word it draws every drawn
// location's u for the 64 shots (Philox4x32-10, one block per l/4, in plain
// loops over the 64 lanes that the compiler turns into SIMD), turns the draws
// into per-variable 64-bit masks by the exact integer thresholds, and XORs
// each nonzero mask into the rows of its variable's column of M.  It reads
// the host model only (column lists, location table, channels), so it is a
// second, independent evaluator of what the device model encodes.
#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "sp_internal.hpp"

namespace sp {
int set_error(int code, const std::string& msg);
}

using sp::set_error;

namespace {

constexpr uint32_t kM0 = 0xD2511F53u;   // Philox4x32 round multipliers
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;   // Philox key increments
constexpr uint32_t kW1 = 0xBB67AE85u;

// One drawn location of a Philox block.
struct Slot {
  uint32_t word;    // l mod 4: which output word of the block it reads
  uint32_t tm1;     // T_m - 1: the location fires when u <= tm1
  uint32_t var0;    // its first variable (column of M)
  uint32_t nbits;   // code bits (variables) of the location
  uint32_t m;       // non-identity codes of its channel
  uint32_t T[16];   // T_1..T_{m-1} (a fired u picks 1 + #{k < m : T_k <= u})
};

struct Block {
  uint32_t blk;          // l / 4
  uint32_t s0, s1;       // its slots [s0, s1)
};

struct Plan {
  std::vector<Block> blocks;
  std::vector<Slot> slots;
};

Plan make_plan(const sp_model& m) {
  Plan P;
  int64_t cur = -1;
  for (uint32_t l = 0; l < m.n_locs; ++l) {
    if (!sp::loc_drawn(m, l)) continue;
    const sp::Channel& ch = m.channels[m.loc_chan[l]];
    if ((int64_t)(l >> 2) != cur) {
      cur = l >> 2;
      P.blocks.push_back(Block{l >> 2, (uint32_t)P.slots.size(), (uint32_t)P.slots.size()});
    }
    Slot s{};
    s.word = l & 3u;
    s.tm1 = (uint32_t)(ch.T[ch.m] - 1);   // T_m >= 1 for a drawn location
    s.var0 = (uint32_t)m.loc_var0[l];
    s.nbits = sp::loc_bits(m.loc_kind[l]);
    s.m = ch.m;
    for (uint32_t k = 1; k < ch.m && k < 16; ++k) s.T[k] = (uint32_t)ch.T[k];
    P.slots.push_back(s);
    P.blocks.back().s1 = (uint32_t)P.slots.size();
  }
  return P;
}

// 64 lanes of one Philox block: lane i draws for counter (blk, lo[i], hi[i], 0).
struct Lanes {
  alignas(64) uint32_t u[4][64];
};

// Philox4x32-10 (Salmon et al., SC'11) over 64 counters (blk, lo[i], hi[i],
// 0) under key (key0, key1), then the fire masks of the requested output
// words: bit i of fire[w] is u[w][i] <= tm1[w].  Three versions with the
// same result: AVX-512, AVX2 and plain C++, picked once by the CPU's
// features.  A round multiplies words 0 and 2 by their constants (32 x 32 ->
// 64 bits: the SIMD versions form the products of even and odd 32-bit lanes
// separately and interleave their halves) and XORs the high halves with
// words 1 and 3 and the round key.
void draw_block_plain(uint32_t blk, const uint32_t* lo, const uint32_t* hi, uint32_t key0, uint32_t key1,
                      const uint32_t* tm1, uint32_t want, Lanes& out, uint64_t* fire) {
  for (int i = 0; i < 64; ++i) {
    uint32_t c0 = blk, c1 = lo[i], c2 = hi[i], c3 = 0, k0 = key0, k1 = key1;
    for (int r = 0; r < 10; ++r) {
      const uint64_t p0 = (uint64_t)kM0 * c0;
      const uint64_t p1 = (uint64_t)kM1 * c2;
      const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
      const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
      c1 = (uint32_t)p1;
      c3 = (uint32_t)p0;
      c0 = n0;
      c2 = n2;
      k0 += kW0;
      k1 += kW1;
    }
    out.u[0][i] = c0;
    out.u[1][i] = c1;
    out.u[2][i] = c2;
    out.u[3][i] = c3;
  }
  for (uint32_t w = 0; w < 4; ++w) {
    if (!((want >> w) & 1u)) continue;
    uint64_t f = 0;
    for (int i = 0; i < 64; ++i) f |= (uint64_t)(out.u[w][i] <= tm1[w]) << i;
    fire[w] = f;
  }
}

__attribute__((target("avx512f"))) void draw_block_avx512(uint32_t blk, const uint32_t* lo, const uint32_t* hi,
                                                          uint32_t key0, uint32_t key1, const uint32_t* tm1,
                                                          uint32_t want, Lanes& out, uint64_t* fire) {
  constexpr int G = 4;   // groups of 16 lanes, advanced together for independent chains
  const __m512i m0 = _mm512_set1_epi64(kM0), m1 = _mm512_set1_epi64(kM1);
  __m512i c0[G], c1[G], c2[G], c3[G];
  for (int g = 0; g < G; ++g) {
    c0[g] = _mm512_set1_epi32((int)blk);
    c1[g] = _mm512_loadu_si512(lo + 16 * g);
    c2[g] = _mm512_loadu_si512(hi + 16 * g);
    c3[g] = _mm512_setzero_si512();
  }
  uint32_t k0 = key0, k1 = key1;
  for (int r = 0; r < 10; ++r) {
    const __m512i vk0 = _mm512_set1_epi32((int)k0), vk1 = _mm512_set1_epi32((int)k1);
    for (int g = 0; g < G; ++g) {
      const __m512i e0 = _mm512_mul_epu32(c0[g], m0), o0 = _mm512_mul_epu32(_mm512_srli_epi64(c0[g], 32), m0);
      const __m512i e1 = _mm512_mul_epu32(c2[g], m1), o1 = _mm512_mul_epu32(_mm512_srli_epi64(c2[g], 32), m1);
      const __m512i lo0 = _mm512_mask_blend_epi32(0xAAAA, e0, _mm512_slli_epi64(o0, 32));
      const __m512i hi0 = _mm512_mask_blend_epi32(0xAAAA, _mm512_srli_epi64(e0, 32), o0);
      const __m512i lo1 = _mm512_mask_blend_epi32(0xAAAA, e1, _mm512_slli_epi64(o1, 32));
      const __m512i hi1 = _mm512_mask_blend_epi32(0xAAAA, _mm512_srli_epi64(e1, 32), o1);
      const __m512i n0 = _mm512_ternarylogic_epi32(hi1, c1[g], vk0, 0x96);   // a ^ b ^ c
      const __m512i n2 = _mm512_ternarylogic_epi32(hi0, c3[g], vk1, 0x96);
      c1[g] = lo1;
      c3[g] = lo0;
      c0[g] = n0;
      c2[g] = n2;
    }
    k0 += kW0;
    k1 += kW1;
  }
  for (int g = 0; g < G; ++g) {
    _mm512_storeu_si512(out.u[0] + 16 * g, c0[g]);
    _mm512_storeu_si512(out.u[1] + 16 * g, c1[g]);
    _mm512_storeu_si512(out.u[2] + 16 * g, c2[g]);
    _mm512_storeu_si512(out.u[3] + 16 * g, c3[g]);
  }
  const __m512i* words[4] = {c0, c1, c2, c3};
  for (uint32_t w = 0; w < 4; ++w) {
    if (!((want >> w) & 1u)) continue;
    const __m512i t = _mm512_set1_epi32((int)tm1[w]);
    uint64_t f = 0;
    for (int g = 0; g < G; ++g) f |= (uint64_t)_mm512_cmple_epu32_mask(words[w][g], t) << (16 * g);
    fire[w] = f;
  }
}

__attribute__((target("avx2"))) void draw_block_avx2(uint32_t blk, const uint32_t* lo, const uint32_t* hi,
                                                     uint32_t key0, uint32_t key1, const uint32_t* tm1,
                                                     uint32_t want, Lanes& out, uint64_t* fire) {
  constexpr int G = 8;   // groups of 8 lanes
  const __m256i m0 = _mm256_set1_epi64x(kM0), m1 = _mm256_set1_epi64x(kM1);
  __m256i c0[G], c1[G], c2[G], c3[G];
  for (int g = 0; g < G; ++g) {
    c0[g] = _mm256_set1_epi32((int)blk);
    c1[g] = _mm256_loadu_si256(reinterpret_cast<const __m256i*>(lo + 8 * g));
    c2[g] = _mm256_loadu_si256(reinterpret_cast<const __m256i*>(hi + 8 * g));
    c3[g] = _mm256_setzero_si256();
  }
  uint32_t k0 = key0, k1 = key1;
  for (int r = 0; r < 10; ++r) {
    const __m256i vk0 = _mm256_set1_epi32((int)k0), vk1 = _mm256_set1_epi32((int)k1);
    for (int g = 0; g < G; ++g) {
      const __m256i e0 = _mm256_mul_epu32(c0[g], m0), o0 = _mm256_mul_epu32(_mm256_srli_epi64(c0[g], 32), m0);
      const __m256i e1 = _mm256_mul_epu32(c2[g], m1), o1 = _mm256_mul_epu32(_mm256_srli_epi64(c2[g], 32), m1);
      const __m256i lo0 = _mm256_blend_epi32(e0, _mm256_slli_epi64(o0, 32), 0xAA);
      const __m256i hi0 = _mm256_blend_epi32(_mm256_srli_epi64(e0, 32), o0, 0xAA);
      const __m256i lo1 = _mm256_blend_epi32(e1, _mm256_slli_epi64(o1, 32), 0xAA);
      const __m256i hi1 = _mm256_blend_epi32(_mm256_srli_epi64(e1, 32), o1, 0xAA);
      const __m256i n0 = _mm256_xor_si256(_mm256_xor_si256(hi1, c1[g]), vk0);
      const __m256i n2 = _mm256_xor_si256(_mm256_xor_si256(hi0, c3[g]), vk1);
      c1[g] = lo1;
      c3[g] = lo0;
      c0[g] = n0;
      c2[g] = n2;
    }
    k0 += kW0;
    k1 += kW1;
  }
  for (int g = 0; g < G; ++g) {
    _mm256_storeu_si256(reinterpret_cast<__m256i*>(out.u[0] + 8 * g), c0[g]);
    _mm256_storeu_si256(reinterpret_cast<__m256i*>(out.u[1] + 8 * g), c1[g]);
    _mm256_storeu_si256(reinterpret_cast<__m256i*>(out.u[2] + 8 * g), c2[g]);
    _mm256_storeu_si256(reinterpret_cast<__m256i*>(out.u[3] + 8 * g), c3[g]);
  }
  // u <= t as unsigned: with the sign bits flipped, not (u > t) as signed
  const __m256i flip = _mm256_set1_epi32((int)0x80000000u);
  const __m256i* words[4] = {c0, c1, c2, c3};
  for (uint32_t w = 0; w < 4; ++w) {
    if (!((want >> w) & 1u)) continue;
    const __m256i t = _mm256_xor_si256(_mm256_set1_epi32((int)tm1[w]), flip);
    uint64_t f = 0;
    for (int g = 0; g < G; ++g) {
      const __m256i gt = _mm256_cmpgt_epi32(_mm256_xor_si256(words[w][g], flip), t);
      const uint32_t m = (uint32_t)_mm256_movemask_ps(_mm256_castsi256_ps(gt));
      f |= (uint64_t)(~m & 0xFFu) << (8 * g);
    }
    fire[w] = f;
  }
}

using DrawFn = void (*)(uint32_t, const uint32_t*, const uint32_t*, uint32_t, uint32_t, const uint32_t*, uint32_t,
                        Lanes&, uint64_t*);

// The widest version the CPU runs.  SYMPHASE_HOST_ISA = plain, avx2 or
// avx512 caps it (the tests compare the three).
DrawFn pick_draw() {
  __builtin_cpu_init();
  const char* cap = std::getenv("SYMPHASE_HOST_ISA");
  const std::string c = cap ? cap : "";
  const bool any = c.empty();
  if ((any || c == "avx512") && __builtin_cpu_supports("avx512f")) return draw_block_avx512;
  if ((any || c == "avx512" || c == "avx2") && __builtin_cpu_supports("avx2")) return draw_block_avx2;
  return draw_block_plain;
}

// Pauli code of a fired draw u: the k with T_{k-1} <= u < T_k.
inline uint32_t code_of(const Slot& s, uint32_t u) {
  uint32_t c = 1;
  for (uint32_t k = 1; k < s.m; ++k) c += s.T[k] <= u ? 1u : 0u;
  return c;
}

struct Job {
  DrawFn draw;
  const sp_model* m;
  const Plan* P;
  uint64_t seed, first_shot, shots;
  uint64_t* out;
  size_t ld;
  uint64_t words;
};

// Samples 64-shot words [w0, w1) with the row accumulators in acc.
void run_words(const Job& J, uint64_t w0, uint64_t w1, std::vector<uint64_t>& acc) {
  const sp_model& m = *J.m;
  const Plan& P = *J.P;
  const uint32_t key0 = (uint32_t)J.seed, key1 = (uint32_t)(J.seed >> 32);
  alignas(64) uint32_t lo[64], hi[64];
  Lanes L;
  for (uint64_t w = w0; w < w1; ++w) {
    for (uint32_t k = 0; k < m.n_meas; ++k) acc[k] = ((m.c_bits[k >> 6] >> (k & 63)) & 1ull) ? ~0ull : 0ull;
    const uint64_t base = J.first_shot + 64 * w;
    for (int i = 0; i < 64; ++i) {
      const uint64_t t = base + (uint64_t)i;
      lo[i] = (uint32_t)t;
      hi[i] = (uint32_t)(t >> 32);
    }
    for (const Block& b : P.blocks) {
      uint32_t tm1[4] = {0, 0, 0, 0}, want = 0;
      for (uint32_t s = b.s0; s < b.s1; ++s) {
        tm1[P.slots[s].word] = P.slots[s].tm1;
        want |= 1u << P.slots[s].word;
      }
      uint64_t fire[4] = {0, 0, 0, 0};
      J.draw(b.blk, lo, hi, key0, key1, tm1, want, L, fire);
      for (uint32_t s = b.s0; s < b.s1; ++s) {
        const Slot& sl = P.slots[s];
        const uint64_t f = fire[sl.word];
        if (!f) continue;
        uint64_t S[4] = {f, 0, 0, 0};   // per code bit: the lanes whose code has it
        if (sl.m > 1) {
          S[0] = 0;
          for (uint64_t x = f; x; x &= x - 1) {
            const uint32_t i = (uint32_t)__builtin_ctzll(x);
            const uint32_t code = code_of(sl, L.u[sl.word][i]);
            for (uint32_t bit = 0; bit < sl.nbits; ++bit)
              if ((code >> bit) & 1u) S[bit] |= 1ull << i;
          }
        }
        for (uint32_t bit = 0; bit < sl.nbits; ++bit) {
          if (!S[bit]) continue;
          const uint32_t v = sl.var0 + bit;
          for (uint32_t e = m.col_ptr[v]; e < m.col_ptr[v + 1]; ++e) acc[m.row_idx[e]] ^= S[bit];
        }
      }
    }
    const uint64_t rem = J.shots - 64 * w;
    const uint64_t valid = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
    for (uint32_t k = 0; k < m.n_meas; ++k) J.out[(size_t)k * J.ld + w] = acc[k] & valid;
  }
}

}  // namespace

extern "C" {

int sp_sample_host(const sp_model* model, uint64_t seed, uint64_t first_shot, uint64_t shots, uint64_t* h_out,
                   size_t ld_words, int n_threads) {
  if (!model) return set_error(SP_E_INVALID, "null model");
  if (shots == 0 || model->n_meas == 0) return SP_OK;
  if (!h_out) return set_error(SP_E_INVALID, "null output");
  const uint64_t words = (shots + 63) / 64;
  if (ld_words < words)
    return set_error(SP_E_INVALID, "ld_words " + std::to_string(ld_words) + " < " + std::to_string(words));
  if (first_shot + shots < first_shot) return set_error(SP_E_INVALID, "shot range overflows 64 bits");
  if (model->n_locs >= (1u << 30)) return set_error(SP_E_LIMIT, "more than 2^30 locations");
  try {
    const Plan P = make_plan(*model);
    Job J{pick_draw(), model, &P, seed, first_shot, shots, h_out, ld_words, words};
    unsigned nt = n_threads > 0 ? (unsigned)n_threads : std::max(1u, std::thread::hardware_concurrency());
    nt = (unsigned)std::min<uint64_t>(std::min(nt, 512u), words);
    constexpr uint64_t kChunk = 4;   // words a thread takes at a time
    std::atomic<uint64_t> next{0};
    // Every thread's row accumulators are allocated here, so that nothing
    // inside a thread can throw.
    std::vector<std::vector<uint64_t>> acc(nt, std::vector<uint64_t>(model->n_meas));
    auto worker = [&](unsigned t) {
      for (;;) {
        const uint64_t w0 = next.fetch_add(kChunk);
        if (w0 >= words) break;
        run_words(J, w0, std::min(words, w0 + kChunk), acc[t]);
      }
    };
    std::vector<std::thread> pool;
    pool.reserve(nt);
    try {
      for (unsigned t = 1; t < nt; ++t) pool.emplace_back(worker, t);
    } catch (const std::system_error&) {
      // fewer threads: the ones started and this one take every word
    }
    worker(0);
    for (std::thread& th : pool) th.join();
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  return SP_OK;
}

}  // extern "C"

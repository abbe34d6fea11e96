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

// Device model: every section lives in the caller's buffer.
struct DevModel {
  const uint32_t* blk_ctr;   // [nb]      Philox block index l/4 of each block
  const uint4* slots;        // [nb][2]   4 slots x (T_m - 1, meta); meta = var0<<8 | (chan+1), 0 = empty
  const uint32_t* chans;     // [nch][16] kind, T_1..T_15
  const uint32_t* col_ptr;   // [n_vars+1]
  const uint32_t* row_idx;   // [nnz]
  const uint64_t* c_mask;    // [ceil(n_meas/64)]
  const uint64_t* dense;     // [n_vars][dense_words] (dense path only)
  uint32_t nb, n_meas, dense_words;
};

struct LaunchArgs {
  DevModel m;
  uint64_t* out;
  uint64_t ld;
  uint64_t first_shot;
  uint64_t shots;
  uint32_t key0, key1;
  uint32_t n_words;
};

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kM0 * c0;
    const uint64_t p1 = (uint64_t)kM1 * c2;
    // three-input XOR in one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kW0;
    k1 += kW1;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// XOR the 64-lane mask s into the slab rows of variable v.
template <int DENSE>
__device__ __forceinline__ void xor_var(const DevModel& m, uint64_t* slab, uint32_t v, uint64_t s, uint32_t lane) {
  if (DENSE) {
    const uint64_t* col = m.dense + (size_t)v * m.dense_words;
    for (uint32_t c = 0; c < m.dense_words; ++c) {
      const uint64_t bits = col[c];
      if (bits == 0) continue;
      if ((bits >> lane) & 1ull) atomicXor((unsigned long long*)&slab[c * 64 + lane], (unsigned long long)s);
    }
  } else {
    const uint32_t lo = m.col_ptr[v], hi = m.col_ptr[v + 1];
    for (uint32_t i = lo + lane; i < hi; i += 64)
      atomicXor((unsigned long long*)&slab[m.row_idx[i]], (unsigned long long)s);
  }
}

// A location fired in the lanes of `fire`: split into code-bit masks and
// evaluate each variable.
template <int DENSE>
__device__ __noinline__ void fire_slot(const DevModel& m, uint64_t* slab, uint32_t u, uint64_t fire, uint32_t meta,
                                       uint32_t lane) {
  const uint32_t ch = (meta & 0xFFu) - 1u;
  const uint32_t var0 = meta >> 8;
  const uint32_t* T = m.chans + ch * 16u;
  const uint32_t kind = T[0];
  if (kind == sp::CH_DEP1) {
    const uint64_t m1 = ballot(u < T[1]), m2 = ballot(u < T[2]);
    const uint64_t bx = m1 ^ m2 ^ fire;   // codes 1, 3
    const uint64_t bz = m1 ^ fire;        // codes 2, 3
    if (bx) xor_var<DENSE>(m, slab, var0, bx, lane);
    if (bz) xor_var<DENSE>(m, slab, var0 + 1, bz, lane);
  } else if (kind == sp::CH_DEP2) {
    uint64_t mk[16];
#pragma unroll
    for (int k = 1; k < 15; ++k) mk[k] = ballot(u < T[k]);
    mk[15] = fire;
    uint64_t b0 = 0, b1 = 0;
#pragma unroll
    for (int k = 1; k <= 15; ++k) {
      b0 ^= mk[k];
      if (k & 1) b1 ^= mk[k];
    }
    const uint64_t b2 = mk[3] ^ mk[7] ^ mk[11] ^ mk[15];
    const uint64_t b3 = mk[7] ^ mk[15];
    if (b0) xor_var<DENSE>(m, slab, var0, b0, lane);
    if (b1) xor_var<DENSE>(m, slab, var0 + 1, b1, lane);
    if (b2) xor_var<DENSE>(m, slab, var0 + 2, b2, lane);
    if (b3) xor_var<DENSE>(m, slab, var0 + 3, b3, lane);
  } else {
    xor_var<DENSE>(m, slab, var0, fire, lane);  // one-variable channels and the coin
  }
}

// blockIdx -> word, keeping consecutive words on one XCD (workgroups are
// dealt round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ uint32_t xcd_word(uint32_t b, uint32_t n) {
  const uint32_t q = n / 8u, r = n % 8u;
  const uint32_t x = b % 8u, i = b / 8u;
  return x * q + min(x, r) + i;
}

template <int DENSE>
__global__ void __launch_bounds__(512) sample_kernel(LaunchArgs a) {
  extern __shared__ uint64_t slab[];
  const DevModel& m = a.m;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = uniform(tid >> 6), n_waves = blockDim.x >> 6;
  const uint32_t w = xcd_word(blockIdx.x, a.n_words);

  for (uint32_t k = tid; k < m.n_meas; k += blockDim.x)
    slab[k] = ((m.c_mask[k >> 6] >> (k & 63u)) & 1ull) ? ~0ull : 0ull;
  __syncthreads();

  const uint64_t shot = a.first_shot + (uint64_t)w * 64u + lane;
  const uint32_t s_lo = (uint32_t)shot, s_hi = (uint32_t)(shot >> 32);

  for (uint32_t b = wave; b < m.nb; b += n_waves) {
    const uint32_t blk = m.blk_ctr[b];
    const uint4 sa = m.slots[2 * b], sb = m.slots[2 * b + 1];
    const uint4 u = philox4x32_10(blk, s_lo, s_hi, 0u, a.key0, a.key1);
    const uint64_t f0 = sa.y ? ballot(u.x <= sa.x) : 0ull;
    const uint64_t f1 = sa.w ? ballot(u.y <= sa.z) : 0ull;
    const uint64_t f2 = sb.y ? ballot(u.z <= sb.x) : 0ull;
    const uint64_t f3 = sb.w ? ballot(u.w <= sb.z) : 0ull;
    if ((f0 | f1 | f2 | f3) == 0ull) continue;
    if (f0) fire_slot<DENSE>(m, slab, u.x, f0, sa.y, lane);
    if (f1) fire_slot<DENSE>(m, slab, u.y, f1, sa.w, lane);
    if (f2) fire_slot<DENSE>(m, slab, u.z, f2, sb.y, lane);
    if (f3) fire_slot<DENSE>(m, slab, u.w, f3, sb.w, lane);
  }
  __syncthreads();

  const uint64_t rem = a.shots - (uint64_t)w * 64u;
  const uint64_t valid = rem >= 64u ? ~0ull : ((1ull << rem) - 1ull);
  uint64_t* col = a.out + w;
  for (uint32_t k = tid; k < m.n_meas; k += blockDim.x) col[(size_t)k * a.ld] = slab[k] & valid;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t blk_ctr, slots, chans, col_ptr, row_idx, c_mask, dense, total;
  uint32_t nb, nch, dense_words;
};

// Drawn locations grouped by Philox block (l/4); blocks without a drawn
// location are left out.
struct Blocks {
  std::vector<uint32_t> ctr;
  std::vector<uint32_t> slots;  // 8 words per block
};

Blocks build_blocks(const sp_model& m) {
  Blocks B;
  int64_t cur = -1;
  for (uint32_t l = 0; l < m.n_locs; ++l) {
    const int32_t ch = m.loc_chan[l];
    if (ch < 0) continue;
    const sp::Channel& c = m.channels[ch];
    const uint64_t Tm = c.T[c.m];
    if (Tm == 0) continue;  // never fires
    const int64_t blk = l >> 2;
    if (blk != cur) {
      B.ctr.push_back((uint32_t)blk);
      B.slots.insert(B.slots.end(), 8, 0u);
      cur = blk;
    }
    uint32_t* s = &B.slots[B.slots.size() - 8 + 2 * (l & 3u)];
    s[0] = (uint32_t)(Tm - 1);
    s[1] = ((uint32_t)m.loc_var0[l] << 8) | (uint32_t)(ch + 1);
  }
  return B;
}

int choose_path(const sp_model& m, int path) {
  if (path != SP_PATH_AUTO) return path;
  // Dense costs ceil(n_meas/64) LDS operations per fired variable, sparse
  // ceil(|column|/64) plus a dependent index load: pick dense only when the
  // columns are long compared with the slab.
  const double avg = m.n_vars ? (double)m.row_idx.size() / m.n_vars : 0.0;
  return (avg * 4.0 > (double)m.n_meas) ? SP_PATH_DENSE : SP_PATH_SPARSE;
}

Layout plan(const sp_model& m, int path, uint32_t nb) {
  Layout L{};
  L.nb = nb;
  L.nch = (uint32_t)m.channels.size();
  L.dense_words = (m.n_meas + 63) / 64;
  size_t off = 0;
  L.blk_ctr = off; off = align256(off + sizeof(uint32_t) * std::max<size_t>(nb, 1));
  L.slots = off;   off = align256(off + 32 * std::max<size_t>(nb, 1));
  L.chans = off;   off = align256(off + 64 * (size_t)L.nch);
  L.col_ptr = off; off = align256(off + sizeof(uint32_t) * (m.n_vars + 1));
  L.row_idx = off; off = align256(off + sizeof(uint32_t) * std::max<size_t>(m.row_idx.size(), 1));
  L.c_mask = off;  off = align256(off + 8 * std::max<size_t>(L.dense_words, 1));
  L.dense = off;
  if (path == SP_PATH_DENSE) off = align256(off + 8 * (size_t)m.n_vars * L.dense_words);
  L.total = off;
  return L;
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return set_error(SP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

struct sp_dmodel {
  DevModel m;
  int path;
  int device;
  sp_dims dims;
};

extern "C" {

int sp_model_device_bytes(const sp_model* model, int path, size_t* bytes) {
  if (!model || !bytes) return set_error(SP_E_INVALID, "null argument");
  if (path < SP_PATH_AUTO || path > SP_PATH_DENSE) return set_error(SP_E_INVALID, "unknown path");
  try {
    Blocks B = build_blocks(*model);
    *bytes = plan(*model, choose_path(*model, path), (uint32_t)B.ctr.size()).total;
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  return SP_OK;
}

int sp_model_upload(const sp_model* model, int path, void* d_buf, size_t buf_bytes, void* stream, sp_dmodel** out) {
  if (!model || !d_buf || !out) return set_error(SP_E_INVALID, "null argument");
  *out = nullptr;
  if (path < SP_PATH_AUTO || path > SP_PATH_DENSE) return set_error(SP_E_INVALID, "unknown path");
  if (((uintptr_t)d_buf & 255u) != 0) return set_error(SP_E_INVALID, "device buffer must be 256-byte aligned");
  if (model->channels.size() > 255) return set_error(SP_E_LIMIT, "more than 255 distinct channels");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  int lds_max = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if ((size_t)model->n_meas * 8 > (size_t)lds_max)
    return set_error(SP_E_LIMIT, "n_meas " + std::to_string(model->n_meas) + " needs " +
                                     std::to_string((size_t)model->n_meas * 8) + " bytes of LDS; the device allows " +
                                     std::to_string(lds_max));
  const int p = choose_path(*model, path);
  std::vector<uint8_t> host;
  Layout L;
  try {
    Blocks B = build_blocks(*model);
    L = plan(*model, p, (uint32_t)B.ctr.size());
    if (buf_bytes < L.total)
      return set_error(SP_E_INVALID, "device buffer of " + std::to_string(buf_bytes) + " bytes, need " +
                                         std::to_string(L.total));
    host.assign(L.total, 0);
    if (!B.ctr.empty()) {
      std::memcpy(&host[L.blk_ctr], B.ctr.data(), 4 * B.ctr.size());
      std::memcpy(&host[L.slots], B.slots.data(), 4 * B.slots.size());
    }
    for (uint32_t c = 0; c < L.nch; ++c) {
      uint32_t* t = reinterpret_cast<uint32_t*>(&host[L.chans + 64 * (size_t)c]);
      const sp::Channel& ch = model->channels[c];
      t[0] = ch.kind;
      for (uint32_t k = 1; k < 16; ++k) t[k] = (uint32_t)std::min<uint64_t>(ch.T[k], 0xFFFFFFFFull);
    }
    std::memcpy(&host[L.col_ptr], model->col_ptr.data(), 4 * model->col_ptr.size());
    if (!model->row_idx.empty()) std::memcpy(&host[L.row_idx], model->row_idx.data(), 4 * model->row_idx.size());
    std::memcpy(&host[L.c_mask], model->c_bits.data(), 8 * L.dense_words);
    if (p == SP_PATH_DENSE) {
      uint64_t* d = reinterpret_cast<uint64_t*>(&host[L.dense]);
      for (uint32_t j = 0; j < model->n_vars; ++j)
        for (uint32_t i = model->col_ptr[j]; i < model->col_ptr[j + 1]; ++i) {
          const uint32_t k = model->row_idx[i];
          d[(size_t)j * L.dense_words + (k >> 6)] |= 1ull << (k & 63);
        }
    }
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(d_buf, host.data(), L.total, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));

  auto* dm = new (std::nothrow) sp_dmodel();
  if (!dm) return set_error(SP_E_NOMEM, "out of host memory");
  const uint8_t* base = (const uint8_t*)d_buf;
  dm->m.blk_ctr = (const uint32_t*)(base + L.blk_ctr);
  dm->m.slots = (const uint4*)(base + L.slots);
  dm->m.chans = (const uint32_t*)(base + L.chans);
  dm->m.col_ptr = (const uint32_t*)(base + L.col_ptr);
  dm->m.row_idx = (const uint32_t*)(base + L.row_idx);
  dm->m.c_mask = (const uint64_t*)(base + L.c_mask);
  dm->m.dense = p == SP_PATH_DENSE ? (const uint64_t*)(base + L.dense) : nullptr;
  dm->m.nb = L.nb;
  dm->m.n_meas = model->n_meas;
  dm->m.dense_words = L.dense_words;
  dm->path = p;
  dm->device = dev;
  sp_model_dims(model, &dm->dims);
  *out = dm;
  return SP_OK;
}

void sp_dmodel_free(sp_dmodel* dm) { delete dm; }

int sp_dmodel_dims(const sp_dmodel* dm, sp_dims* out) {
  if (!dm || !out) return set_error(SP_E_INVALID, "null argument");
  *out = dm->dims;
  return SP_OK;
}

int sp_sample(const sp_dmodel* dm, uint64_t seed, uint64_t first_shot, uint64_t shots, uint64_t* d_out,
              size_t ld_words, void* stream) {
  if (!dm) return set_error(SP_E_INVALID, "null model");
  if (shots == 0 || dm->m.n_meas == 0) return SP_OK;
  if (!d_out) return set_error(SP_E_INVALID, "null output");
  if (((uintptr_t)d_out & 7u) != 0) return set_error(SP_E_INVALID, "output must be 8-byte aligned");
  const uint64_t words = (shots + 63) / 64;
  if (ld_words < words) return set_error(SP_E_INVALID, "ld_words " + std::to_string(ld_words) + " < " + std::to_string(words));
  if (words > 0x7FFFFFFFull) return set_error(SP_E_LIMIT, "too many shots for one launch");
  if (first_shot + shots < first_shot) return set_error(SP_E_INVALID, "shot range overflows 64 bits");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != dm->device) return set_error(SP_E_INVALID, "current device differs from the model's device");

  LaunchArgs a;
  a.m = dm->m;
  a.out = d_out;
  a.ld = ld_words;
  a.first_shot = first_shot;
  a.shots = shots;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.n_words = (uint32_t)words;
  const size_t lds = (size_t)dm->m.n_meas * 8;
  const unsigned threads = 512;
  hipStream_t s = (hipStream_t)stream;
  static std::once_flag once[2];
  if (dm->path == SP_PATH_DENSE) {
    std::call_once(once[1], [] { (void)hipFuncSetAttribute((const void*)sample_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); });
    hipLaunchKernelGGL(sample_kernel<1>, dim3((unsigned)words), dim3(threads), lds, s, a);
  } else {
    std::call_once(once[0], [] { (void)hipFuncSetAttribute((const void*)sample_kernel<0>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); });
    hipLaunchKernelGGL(sample_kernel<0>, dim3((unsigned)words), dim3(threads), lds, s, a);
  }
  HIP_TRY(hipGetLastError());
  return SP_OK;
}

}  // extern "C"

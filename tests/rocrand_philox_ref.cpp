// Third opinion for the Philox4x32-10 block function: calls rocRAND's
// host-callable engine (header-only use of the installed library).
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) and prints the four output words.
// rocrand_init(seed, subsequence, 0) keys the engine with the 64-bit seed and
// puts the subsequence in the high 64 bits of the counter; skipahead(offset)
// adds offset/4 to the low 64 bits; rocrand4 returns the block at the counter.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long block = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, subseq, 0ull, &st);
    // Advance by `block` blocks; each skip moves offset/4 blocks and the
    // offset argument is 64-bit, so go in four quarters plus a remainder.
    for (int i = 0; i < 4; i++) skipahead(4ull * (block >> 2), &st);
    skipahead(4ull * (block & 3ull), &st);
    uint4 v = rocrand4(&st);
    std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}

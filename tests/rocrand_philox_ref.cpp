// Test-only second implementation of Philox4x32-10: rocRAND's header engine,
// driven on the host.  Used by the oracle's pin tests as an independent
// library routine; never linked into the oracle or the GPU library.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" void rocrand_philox_ref(const uint32_t* ctr, const uint32_t* key,
                                   uint32_t* out, int n)
{
    for (int k = 0; k < n; ++k) {
        unsigned long long seed = (unsigned long long)key[2 * k] |
                                  ((unsigned long long)key[2 * k + 1] << 32);
        // rocRAND places the 64-bit draw offset/4 in counter words 0-1 and the
        // subsequence in words 2-3; offset must stay below 2^64.
        unsigned long long off = (((unsigned long long)ctr[4 * k + 1] << 32) | ctr[4 * k]) * 4ull;
        unsigned long long sub = ((unsigned long long)ctr[4 * k + 3] << 32) | ctr[4 * k + 2];
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 r = e.next4();
        out[4 * k] = r.x; out[4 * k + 1] = r.y; out[4 * k + 2] = r.z; out[4 * k + 3] = r.w;
    }
}

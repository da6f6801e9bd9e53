// Independent Philox4x32-10 reference for the oracle's pin: rocRAND's
// header-only engine (public source under /opt/rocm/include/rocrand),
// compiled for the host.  Test infrastructure only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" void ref_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out) {
    // The engine keys with the 64-bit seed (lo word = key 0); the subsequence
    // sets counter words 2-3 and the offset (in 32-bit outputs, four per
    // block) sets counter words 0-1.
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)ctr[2] | ((unsigned long long)ctr[3] << 32);
    unsigned long long blk = (unsigned long long)ctr[0] | ((unsigned long long)ctr[1] << 32);
    rocrand_device::philox4x32_10_engine e(seed, sub, 0);
    // advance the block counter in two halves to avoid 4*blk overflow
    if (blk) {
        e.discard(4ull * (blk & 0xFFFFFFFFull));
        for (unsigned i = 0; i < 4; ++i) e.discard(4ull * ((blk >> 32) << 30));
    }
    uint4 r = e.next4();
    out[0] = r.x; out[1] = r.y; out[2] = r.z; out[3] = r.w;
}

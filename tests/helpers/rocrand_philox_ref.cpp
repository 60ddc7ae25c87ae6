// Host-side access to rocRAND's Philox4x32-10 round function, used only by
// tests to pin the oracle's (and the GPU library's) Philox against an
// independent library implementation of the same published generator.
#include <rocrand/rocrand_philox4x32_10.h>

namespace {
struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};
}  // namespace

extern "C" void ref_philox4x32_10(const unsigned* ctr, const unsigned* key, unsigned* out, long n)
{
    Engine e;
    for (long i = 0; i < n; i++) {
        uint4 c = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        uint2 k = {key[2 * i], key[2 * i + 1]};
        uint4 r = e.apply(c, k);
        out[4 * i] = r.x;
        out[4 * i + 1] = r.y;
        out[4 * i + 2] = r.z;
        out[4 * i + 3] = r.w;
    }
}

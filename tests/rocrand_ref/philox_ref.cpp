// Host build of rocRAND's Philox4x32-10 engine (the ROCm image's own source
// header), exposed as one C function: the ten-round bijection of a 128-bit
// counter under a 64-bit key.  Test infrastructure: it pins the oracle's
// Philox4x32-10 bitwise to an implementation written by others.
#include <rocrand/rocrand_philox4x32_10.h>

#include <stdint.h>

namespace {
// ten_rounds is a protected member of the engine; a derived class reaches it
struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 bijection(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};
}  // namespace

extern "C" void ref_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count) {
    Probe p;
    for (int64_t i = 0; i < count; ++i) {
        uint4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        uint2 k{key[2 * i], key[2 * i + 1]};
        uint4 r = p.bijection(c, k);
        out[4 * i] = r.x;
        out[4 * i + 1] = r.y;
        out[4 * i + 2] = r.z;
        out[4 * i + 3] = r.w;
    }
}

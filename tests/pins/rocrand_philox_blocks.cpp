// Pin helper for the oracle's Philox4x32-10: evaluates rocRAND's own block
// function (host build of rocRAND's header-only engine) on the (counter, key)
// pairs read from stdin, one "c0 c1 c2 c3 k0 k1" line each, and prints the four
// output words per line.  Test infrastructure; not part of any library.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

// ten_rounds is a protected member of the engine; a derived class exposes it.
struct block_engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    block_engine eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr = make_uint4(c0, c1, c2, c3);
        uint2 key = make_uint2(k0, k1);
        uint4 r = eng.block(ctr, key);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}

// Independent Philox4x32-10 block from rocRAND's host/device engine, used only
// to pin the oracle's own Philox4x32-10 against a second implementation.
// Arguments come in groups of four: seed m r t.  The engine is started at
// subsequence (t << 32 | r) and offset 4 m, i.e. at counter (lo m, hi m, r, t)
// with key (lo seed, hi seed); the first 4-word block is printed.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
    for (int a = 1; a + 3 < argc; a += 4) {
        unsigned long long seed = std::strtoull(argv[a], nullptr, 0);
        unsigned long long m = std::strtoull(argv[a + 1], nullptr, 0);
        unsigned long long r = std::strtoull(argv[a + 2], nullptr, 0);
        unsigned long long t = std::strtoull(argv[a + 3], nullptr, 0);
        rocrand_device::philox4x32_10_engine eng(seed, (t << 32) | r, 4ull * m);
        uint4 v = eng.next4();
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}

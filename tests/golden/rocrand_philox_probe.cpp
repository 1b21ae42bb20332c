// Prints Philox4x32-10 outputs of rocRAND's host-usable engine for
// (seed, subsequence, offset) triples read from stdin.  Used only by
// tests/test_oracle_rng.py as an implementation independent of the oracle.
// rocRAND maps seed -> key, subsequence -> counter words 2..3 and
// offset/4 -> counter words 0..1.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llx %llx %llx", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}

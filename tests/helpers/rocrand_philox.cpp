// Prints rocRAND's Philox4x32-10 output for counters read from stdin (host execution only).
// Input lines: c0 c1 c2 c3 k0 k1 (decimal).  The engine's ten-round function is reached
// through a derived class, so the raw bijection Philox(counter, key) is evaluated by
// rocRAND's own code.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 eval(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main() {
    unsigned int c0, c1, c2, c3, k0, k1;
    Probe p;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c;
        c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k;
        k.x = k0; k.y = k1;
        uint4 v = p.eval(c, k);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}

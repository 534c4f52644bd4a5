// Drives daqk::Arena from a list of operations on stdin (CPU test helper).
//   a <bytes>   -> prints the offset (or -1)
//   r <offset>  -> prints 1 / 0
//   s           -> prints in_use peak largest_free free_ranges live_blocks
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "arena.h"

int main(int argc, char **argv) {
    daqk::Arena a(argc > 1 ? strtoull(argv[1], nullptr, 10) : 0);
    char op[8];
    unsigned long long v = 0;
    while (scanf("%7s", op) == 1) {
        if (op[0] == 'a' && scanf("%llu", &v) == 1) {
            printf("%lld\n", (long long)a.alloc(v));
        } else if (op[0] == 'r' && scanf("%llu", &v) == 1) {
            printf("%d\n", a.release(v) ? 1 : 0);
        } else if (op[0] == 's') {
            printf("%llu %llu %llu %zu %zu\n", (unsigned long long)a.in_use(), (unsigned long long)a.peak(),
                   (unsigned long long)a.largest_free(), a.free_ranges(), a.live_blocks());
        }
    }
    return 0;
}

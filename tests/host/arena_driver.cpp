// Host-only driver for au::Arena (the server's first-fit allocator): reads
// commands from stdin and prints the allocator's answers, so the test can
// compare them with a reference model.
//   init <size>            -> "ok"
//   alloc <bytes>          -> "ok <offset>" | "full"
//   free <offset> <bytes>  -> "ok"
//   stat                   -> "<in_use> <peak> <size>"
#include <cstdio>
#include <cstring>
#include <string>

#include "au_arena.h"

int main()
{
    au::Arena a;
    char cmd[32];
    while (std::scanf("%31s", cmd) == 1) {
        if (!std::strcmp(cmd, "init")) {
            unsigned long long n;
            std::scanf("%llu", &n);
            a.init(n);
            std::printf("ok\n");
        } else if (!std::strcmp(cmd, "alloc")) {
            unsigned long long n;
            std::scanf("%llu", &n);
            size_t off = 0;
            if (a.alloc(n, &off)) std::printf("ok %llu\n", (unsigned long long)off);
            else std::printf("full\n");
        } else if (!std::strcmp(cmd, "free")) {
            unsigned long long o, n;
            std::scanf("%llu %llu", &o, &n);
            a.release(o, n);
            std::printf("ok\n");
        } else if (!std::strcmp(cmd, "stat")) {
            std::printf("%llu %llu %llu\n", (unsigned long long)a.in_use(), (unsigned long long)a.peak(),
                        (unsigned long long)a.size());
        }
    }
    return 0;
}

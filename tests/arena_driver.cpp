// Drives the quote server's arena allocator from a script of operations on
// stdin ("a <bytes>" allocate, "f <offset> <bytes>" free, "s" report) and
// prints one line per operation.  Compiled and run by test_server_cpu.py.
#include <cstdio>
#include <cstring>

#include "arena.h"

int main(int argc, char **argv) {
    size_t total = argc > 1 ? static_cast<size_t>(atoll(argv[1])) : 1000;
    ara::Arena a;
    a.init(total);
    char op[8];
    while (scanf("%7s", op) == 1) {
        if (!strcmp(op, "a")) {
            size_t n;
            if (scanf("%zu", &n) != 1) return 2;
            size_t off = 0;
            if (a.alloc(n, &off)) printf("ok %zu\n", off);
            else printf("full\n");
        } else if (!strcmp(op, "f")) {
            size_t off, n;
            if (scanf("%zu %zu", &off, &n) != 2) return 2;
            a.release(off, n);
            printf("freed\n");
        } else if (!strcmp(op, "s")) {
            printf("free %zu\n", a.free_bytes());
        }
    }
    return 0;
}

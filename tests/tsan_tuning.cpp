// Two threads set and read back their kernel-shape tunings concurrently
// through the C ABI (lrq_set_tuning / lrq_get_tuning).  Built with
// -fsanitize=thread against the library's host-only translation unit by
// tests/test_abi_host.py: a data race on the tuning state makes the sanitizer
// report it and exit non-zero, and a thread that reads another thread's
// setting fails the check below.
#include <cstdio>
#include <thread>

#include "lrq.h"

static int run(int which, int *bad) {
    const lrq_tuning mine = which ? lrq_tuning{32, 4, 4096, 1} : lrq_tuning{16, 8, 1024, 0};
    for (int it = 0; it < 20000; ++it) {
        if (lrq_set_tuning(it % 3 == 2 ? nullptr : &mine) != LRQ_OK) { ++*bad; return 1; }
        lrq_tuning got{};
        if (lrq_get_tuning(&got) != LRQ_OK) { ++*bad; return 1; }
        const lrq_tuning want = it % 3 == 2 ? lrq_tuning{8, 8, 2048, 0} : mine;
        if (got.plcp_chunk != want.plcp_chunk || got.llr_waves != want.llr_waves ||
            got.lr_tile != want.lr_tile || got.fuse_filter != want.fuse_filter)
            ++*bad;
    }
    return 0;
}

int main() {
    int bad0 = 0, bad1 = 0;
    std::thread a(run, 0, &bad0), b(run, 1, &bad1);
    a.join();
    b.join();
    std::printf("mismatches: %d %d\n", bad0, bad1);
    return bad0 || bad1 ? 1 : 0;
}

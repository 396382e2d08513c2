/* A plain C99 consumer of include/lrq.h: compiles against the header alone,
 * links liblrq.so, and exercises the host-side calls (no GPU needed). */
#include <stdio.h>
#include <string.h>

#include "lrq.h"

#define CHECK(cond)                                                      \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "failed: %s (line %d): %s\n", #cond,          \
                    __LINE__, lrq_last_error());                         \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(void) {
    const char *text = "mississippi";
    const int32_t want[11] = {10, 7, 4, 1, 0, 9, 8, 6, 3, 5, 2}; /* Table 1, 0-based */
    int32_t sa[11];
    size_t bytes = 0;
    lrq_tuning tu;
    lrq_rec rec = {-1, 0};
    int64_t off[3] = {0, 4, 11};
    int32_t sa2[11];

    CHECK(lrq_version() == LRQ_API_VERSION);
    CHECK(strcmp(lrq_status_str(LRQ_OK), "ok") == 0);
    CHECK(lrq_build_sa_host((const uint8_t *)text, 11, sa) == LRQ_OK);
    CHECK(memcmp(sa, want, sizeof want) == 0);
    CHECK(lrq_build_sa_host_batch((const uint8_t *)text, off, 2, sa2) == LRQ_OK);
    CHECK(sa2[0] == 1 && sa2[1] == 0);                       /* "miss": i < iss < m < ss ... */
    CHECK(lrq_scratch_bytes(1 << 20, 1, &bytes) == LRQ_OK && bytes > 0);
    CHECK(lrq_scratch_bytes(-1, 1, &bytes) == LRQ_EINVAL);
    CHECK(lrq_get_tuning(&tu) == LRQ_OK && tu.lr_tile == 2048 && tu.fuse_filter == 0);
    tu.lr_tile = 3000;
    CHECK(lrq_set_tuning(&tu) == LRQ_EINVAL);
    CHECK(lrq_set_tuning(NULL) == LRQ_OK);
    CHECK(lrq_rank_scatter(NULL, -1, NULL, 1, NULL, NULL, NULL, 0, NULL) == LRQ_EINVAL);
    CHECK(lrq_lr_leftmost(NULL, NULL, 10, NULL, 1, &rec, NULL, 0, NULL) == LRQ_EINVAL);
    CHECK(lrq_lr_both(NULL, NULL, 10, NULL, 1, NULL, NULL, NULL, 0, NULL, NULL, 0, NULL) == LRQ_EINVAL);
    CHECK(lrq_llr_lengths(NULL, 0, NULL, NULL) == LRQ_OK);
    CHECK(lrq_llr_lengths(NULL, 10, NULL, NULL) == LRQ_EINVAL);
    CHECK(lrq_lr_leftmost_raw(NULL, 10, NULL, 1, 0, &rec, NULL, 0, NULL) == LRQ_EINVAL);
    CHECK(lrq_lr_all_raw(NULL, 10, NULL, 1, 0, NULL, NULL, NULL, 0, NULL, NULL, 0, NULL) == LRQ_EINVAL);
    CHECK(lrq_sa_work_bytes(1 << 20, 1, &bytes) == LRQ_OK && bytes >= (size_t)32 << 20);
    CHECK(lrq_build_sa(NULL, 10, NULL, 1, NULL, NULL, 0, NULL) == LRQ_EINVAL);
    CHECK(sizeof(lrq_rec) == 8 && sizeof(lrq_string_ref) == 40);
    printf("c abi ok\n");
    return 0;
}

/* Host sanitizer driver for the C ABI (test infrastructure): every entry
 * point's argument checks and host-only calls, which run without a GPU,
 * under AddressSanitizer and UndefinedBehaviorSanitizer. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "kdtree.h"

static int failures = 0;
#define EXPECT(cond) do { if (!(cond)) { printf("failed: %s (line %d)\n", #cond, __LINE__); failures++; } } while (0)

int main(void)
{
    kd_params p;
    memset(&p, 0, sizeof(p));
    p.leaf_size = 32; p.num_subsets = 16; p.fourier_J = 15;
    uint64_t cap = 0, ws = 0;
    for (uint32_t rule = 0; rule < 3; rule++)
        for (uint32_t key = 0; key < 2; key++) {
            p.split_rule = rule; p.key_rule = key;
            EXPECT(kd_tree_bounds(1u << 20, 8, &p, &cap, &ws) == KD_OK);
            EXPECT(cap == 4 * ((1u << 20) / 32) + 64 && ws > 0);
        }
    p.split_rule = 0; p.key_rule = 0;
    EXPECT(kd_tree_bounds(0, 3, &p, &cap, &ws) == KD_EINVAL);
    EXPECT(kd_tree_bounds(100, 0, &p, &cap, &ws) == KD_EINVAL);
    EXPECT(kd_tree_bounds(100, 5000, &p, &cap, &ws) == KD_EINVAL);
    p.leaf_size = 0; EXPECT(kd_tree_bounds(100, 3, &p, &cap, &ws) == KD_EINVAL); p.leaf_size = 32;
    p.num_subsets = 5000; EXPECT(kd_tree_bounds(100, 3, &p, &cap, &ws) == KD_EINVAL); p.num_subsets = 16;
    p.flags = 2; EXPECT(kd_tree_bounds(100, 3, &p, &cap, &ws) == KD_EINVAL); p.flags = 0;
    p.split_rule = 1; p.fourier_J = 0; EXPECT(kd_tree_bounds(100, 3, &p, &cap, &ws) == KD_EINVAL);
    p.split_rule = 0; p.fourier_J = 15;
    EXPECT(kd_tree_bounds(100, 3, NULL, &cap, &ws) == KD_EINVAL);

    /* entry points reject bad arguments before touching the device */
    kd_tree t;
    memset(&t, 0, sizeof(t));
    float dummy[4];
    EXPECT(kd_build(NULL, 10, 1, 10, &p, &t, dummy, 16, NULL) == KD_EINVAL);
    EXPECT(kd_build(dummy, 10, 1, 10, &p, &t, dummy, 16, NULL) == KD_EINVAL);  /* tree arrays missing */
    EXPECT(kd_build_noalloc(dummy, 10, 1, 10, &p, &t, NULL) == KD_EINVAL);
    EXPECT(kd_build_batched(0, NULL, &p, dummy, 16, NULL) == KD_EINVAL);
    EXPECT(kd_batch_bounds(0, NULL, &p, &ws) == KD_EINVAL);
    uint32_t out[4];
    EXPECT(kd_query_leaf(&t, dummy, 1, 1, 1, out, NULL) == KD_EINVAL);
    EXPECT(kd_query_knn(&t, 10, dummy, 1, 1, 1, 4, out, (double *)dummy, NULL) == KD_EINVAL);
    EXPECT(kd_query_box(&t, 10, dummy, dummy, 1, 1, 1, out, NULL, NULL, NULL) == KD_EINVAL);
    EXPECT(kd_global_moments(NULL, 10, 3, 10, 15, NULL, NULL) == KD_EINVAL);
    EXPECT(kd_global_solve(NULL, 3, 15, 6, NULL, NULL) == KD_EINVAL);
    EXPECT(kd_global_counts(NULL, 10, 3, 10, NULL, 6, NULL, NULL) == KD_EINVAL);

    kd_tuning tn, back;
    memset(&tn, 0, sizeof(tn));
    tn.hist_blocks = 7; tn.scatter_blocks = 9; tn.small_blocks = 11;
    EXPECT(kd_set_tuning(&tn) == KD_OK);
    EXPECT(kd_get_tuning(&back) == KD_OK && back.hist_blocks == 7 && back.small_blocks == 11);
    memset(&tn, 0, sizeof(tn));
    EXPECT(kd_set_tuning(&tn) == KD_OK);
    for (int s = -1; s < 9; s++) EXPECT(kd_status_string(s) != NULL);
    EXPECT(kd_version() > 0);
    printf("%s\n", failures ? "FAILED" : "ok");
    return failures != 0;
}

/* Host sanitizer driver for the oracle (test infrastructure): builds trees
 * with every split rule, key rule and subset kind on small random inputs,
 * with ties and signed zeros, under AddressSanitizer and
 * UndefinedBehaviorSanitizer, and checks the structural invariants. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct kdo_params {
    uint32_t leaf_size, max_depth, num_subsets, key_rule, split_rule, fourier_J;
    const uint32_t *pool;
    uint32_t pool_entries, pad_;
    uint64_t seed, node_capacity;
} kdo_params;

int kdo_build(const float *pts, uint64_t n, uint32_t d, uint64_t ld, const kdo_params *p,
              uint32_t *perm, uint32_t *node_begin, uint32_t *node_end, int32_t *node_child,
              uint32_t *node_dim, uint32_t *node_split, uint32_t *node_leaf,
              uint32_t *leaf_node, uint32_t *leaf_offsets, uint64_t *hdr);
uint64_t kdo_check_partition(const float *pts, uint32_t d, uint64_t ld, const uint32_t *perm,
                             uint64_t num_nodes, const uint32_t *node_begin,
                             const uint32_t *node_end, const int32_t *node_child,
                             const uint32_t *node_dim, const uint32_t *node_split);
void kdo_build_batched(uint32_t count, const float *const *pts, const uint64_t *n,
                       const uint32_t *d, const kdo_params *params, void *const *out, int *status);

static uint64_t rng = 88172645463325252ull;
static uint32_t next_u32(void)
{
    rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
    return (uint32_t)(rng >> 11);
}

int main(void)
{
    int failures = 0;
    const uint64_t sizes[] = {1, 2, 3, 31, 33, 200, 4097, 9000};
    uint32_t pool[8 * 4];
    for (int e = 0; e < 8; e++) {
        uint32_t acc = 0;
        pool[e * 4] = 0;
        for (int r = 1; r < 4; r++) { acc += next_u32() >> 3; pool[e * 4 + r] = acc; }
    }
    for (size_t si = 0; si < sizeof(sizes) / sizeof(sizes[0]); si++)
        for (uint32_t d = 1; d <= 5; d += 2)
            for (uint32_t rule = 0; rule < 3; rule++)
                for (uint32_t key = 0; key < 2; key++)
                    for (int usepool = 0; usepool < 2; usepool++) {
                        uint64_t n = sizes[si];
                        float *x = malloc(n * d * sizeof(float));
                        for (uint64_t i = 0; i < n * d; i++) {
                            uint32_t r = next_u32();
                            x[i] = (r % 7 == 0) ? -0.0f : (float)(int)(r % 50) - 25.0f;
                            if (r % 5 == 0) x[i] = (float)r * 1e-7f;
                        }
                        kdo_params p;
                        memset(&p, 0, sizeof(p));
                        p.leaf_size = 1 + next_u32() % 8;
                        p.num_subsets = 4;
                        p.key_rule = key;
                        p.split_rule = rule;
                        p.fourier_J = 15;
                        p.pool = usepool ? pool : NULL;
                        p.pool_entries = usepool ? 8 : 0;
                        p.seed = 5;
                        p.node_capacity = 2 * n + 64;
                        uint64_t cap = p.node_capacity;
                        uint32_t *perm = malloc(n * 4), *nb = malloc(cap * 4), *ne = malloc(cap * 4);
                        int32_t *nc = malloc(cap * 4);
                        uint32_t *nd = malloc(cap * 4), *ns = malloc(cap * 4), *nl = malloc(cap * 4);
                        uint32_t *ln = malloc(cap * 4), *lo = malloc((cap + 1) * 4);
                        uint64_t hdr[7];
                        int st = kdo_build(x, n, d, n, &p, perm, nb, ne, nc, nd, ns, nl, ln, lo, hdr);
                        if (st != 0) { printf("status %d n=%lu\n", st, (unsigned long)n); failures++; }
                        else if (kdo_check_partition(x, d, n, perm, hdr[0], nb, ne, nc, nd, ns) != 0) {
                            printf("partition n=%lu rule=%u\n", (unsigned long)n, rule);
                            failures++;
                        }
                        free(perm); free(nb); free(ne); free(nc); free(nd); free(ns);
                        free(nl); free(ln); free(lo); free(x);
                    }
    /* the batched entry on three trees */
    {
        uint64_t ns[3] = {50, 700, 3};
        uint32_t ds[3] = {2, 3, 1};
        float *px[3];
        kdo_params prm[3];
        void *out[30];
        int st[3];
        for (int k = 0; k < 3; k++) {
            px[k] = malloc(ns[k] * ds[k] * sizeof(float));
            for (uint64_t i = 0; i < ns[k] * ds[k]; i++) px[k][i] = (float)(next_u32() % 100);
            memset(&prm[k], 0, sizeof(prm[k]));
            prm[k].leaf_size = 4; prm[k].num_subsets = 2; prm[k].fourier_J = 15;
            prm[k].split_rule = (uint32_t)k; prm[k].node_capacity = 2 * ns[k] + 64;
            uint64_t cap = prm[k].node_capacity;
            out[10 * k + 0] = malloc(ns[k] * 4);
            for (int a = 1; a < 8; a++) out[10 * k + a] = malloc(cap * 4);
            out[10 * k + 8] = malloc((cap + 1) * 4);
            out[10 * k + 9] = malloc(7 * 8);
        }
        kdo_build_batched(3, (const float *const *)px, ns, ds, prm, out, st);
        for (int k = 0; k < 3; k++) {
            if (st[k] != 0) { printf("batched status %d\n", st[k]); failures++; }
            for (int a = 0; a < 10; a++) free(out[10 * k + a]);
            free(px[k]);
        }
    }
    printf("%s\n", failures ? "FAILED" : "ok");
    return failures != 0;
}

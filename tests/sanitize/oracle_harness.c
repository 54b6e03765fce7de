/* The oracle's construction and query on the CPU under AddressSanitizer and
 * UBSan: for several sizes and the Default, Fast and single-part mod
 * settings, and for byte strings with 64- and 128-bit hashes, the queries of
 * all keys must form a permutation of [0, n). Test infrastructure only. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
static uint64_t sm(uint64_t x) { x += 0x9e3779b97f4a7c15ull; x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull; x = (x ^ (x >> 27)) * 0x94d049bb133111ebull; return x ^ (x >> 31); }
static int check_perm(const uint64_t *out, uint64_t n) {
    char *seen = calloc(n ? n : 1, 1);
    for (uint64_t i = 0; i < n; ++i) { if (out[i] >= n || seen[out[i]]) { free(seen); return 1; } seen[out[i]] = 1; }
    free(seen); return 0;
}
int main(void) {
    int fails = 0;
    uint64_t sizes[] = {1, 2, 3, 17, 100, 1000, 65537, 200000};
    orc_build_cfg cfg = {10, 16};
    for (unsigned si = 0; si < sizeof sizes / sizeof *sizes; ++si) {
        uint64_t n = sizes[si];
        uint64_t *keys = malloc(n * 8), *out = malloc(n * 8);
        for (uint64_t i = 0; i < n; ++i) keys[i] = sm(i * 3 + 5);
        for (int variant = 0; variant < 3; ++variant) {
            orc_params p;
            int rc = variant == 2 ? orc_params_for_single_mod(n, 0.99, 3.5, 0, 0, &p)
                                  : orc_params_for(n, 0.99, variant ? 3.0 : 3.5, variant, 0, 0, &p);
            if (rc) { printf("params n=%llu v=%d rc=%d\n", (unsigned long long)n, variant, rc); ++fails; continue; }
            uint8_t *pil = calloc(p.num_parts * p.buckets_per_part, 1);
            uint64_t *F = calloc(p.remap_len + 1, 8);
            orc_build_stats st;
            rc = orc_build_u64(&p, keys, &cfg, pil, F, &st);
            if (rc) { printf("build n=%llu v=%d rc=%d\n", (unsigned long long)n, variant, rc); ++fails; }
            else {
                uint8_t *clef = calloc(orc_clef_bytes(p.remap_len) + 64, 1);
                if (orc_clef_encode(F, p.remap_len, clef)) { printf("clef n=%llu\n", (unsigned long long)n); ++fails; }
                orc_query_u64(&p, pil, ORC_REMAP_CLEF, clef, keys, n, out);
                if (check_perm(out, n)) { printf("not a permutation n=%llu v=%d\n", (unsigned long long)n, variant); ++fails; }
                free(clef);
            }
            free(pil); free(F);
        }
        free(keys); free(out);
    }
    /* strings, 64- and 128-bit */
    for (int hb = 64; hb <= 128; hb += 64) {
        uint64_t n = 5000, *off = malloc((n + 1) * 8), *out = malloc(n * 8);
        uint8_t *data = calloc(n * 80 + 128, 1); uint64_t pos = 0;
        for (uint64_t i = 0; i < n; ++i) {
            off[i] = pos; uint64_t len = sm(i) % 60;
            for (uint64_t j = 0; j < len; ++j) data[pos++] = (uint8_t)sm(i * 131 + j);
            for (int b = 0; b < 8; ++b) data[pos++] = (uint8_t)(i >> (8 * b));
        }
        off[n] = pos;
        orc_params p; orc_params_for(n, 0.99, 3.5, 0, 0, 0, &p); p.hash_bits = hb;
        uint8_t *pil = calloc(p.num_parts * p.buckets_per_part, 1); uint64_t *F = calloc(p.remap_len + 1, 8);
        orc_build_stats st;
        int rc = orc_build_bytes(&p, data, off, &cfg, pil, F, &st);
        if (rc) { printf("bytes build hb=%d rc=%d\n", hb, rc); ++fails; }
        else {
            orc_query_bytes(&p, pil, ORC_REMAP_PLAIN, F, data, off, n, out);
            if (check_perm(out, n)) { printf("bytes not a permutation hb=%d\n", hb); ++fails; }
        }
        free(off); free(out); free(data); free(pil); free(F);
    }
    printf("oracle asan harness done, %d failures\n", fails);
    return fails != 0;
}

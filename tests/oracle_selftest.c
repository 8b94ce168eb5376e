/*
 * Self-test driver of the CPU oracle for sanitizer builds (AddressSanitizer
 * and UndefinedBehaviorSanitizer): it runs every oracle entry point over
 * seeded inputs of many shapes and checks what the stable sort fixes
 * (keys in order, the payloads a permutation that carries every key, equal
 * keys in input order), so that an out-of-bounds access, a leak or an
 * undefined operation anywhere in the oracle fails the build's test.
 * Built and run by tests/test_oracle_sanitizers.py; not part of any library.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

static int failures = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);               \
            fprintf(stderr, "\n");                      \
            ++failures;                                 \
        }                                               \
    } while (0)

static uint64_t rng_state = 12345;
static uint64_t next_rand(void) { return orc_splitmix64(&rng_state); }

static void fill(uint64_t* x, int64_t n, int kind)
{
    for (int64_t i = 0; i < n; ++i) {
        switch (kind) {
        case 0: x[i] = next_rand(); break;                 /* distinct-ish */
        case 1: x[i] = next_rand() % 3; break;             /* many ties */
        case 2: x[i] = (uint64_t)i / 7; break;             /* sorted */
        case 3: x[i] = (uint64_t)(n - i); break;           /* reversed */
        default: x[i] = (i % 97 == 0) ? next_rand() : (uint64_t)i; break;  /* presorted */
        }
    }
}

/* keys ascending, vals a permutation of 0..n-1 carrying its key, ties in order */
static void check_stable(const uint64_t* orig, const uint64_t* keys, const uint32_t* vals, int64_t n,
                         const char* what)
{
    char* seen = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t i = 0; i < n; ++i) {
        CHECK(vals[i] < (uint64_t)n, "%s: value out of range at %lld", what, (long long)i);
        if (vals[i] >= (uint64_t)n) break;
        CHECK(!seen[vals[i]], "%s: value repeated at %lld", what, (long long)i);
        seen[vals[i]] = 1;
        CHECK(orig[vals[i]] == keys[i], "%s: key not carried at %lld", what, (long long)i);
        if (i > 0) {
            CHECK(keys[i - 1] <= keys[i], "%s: keys out of order at %lld", what, (long long)i);
            if (keys[i - 1] == keys[i]) CHECK(vals[i - 1] < vals[i], "%s: unstable at %lld", what, (long long)i);
        }
    }
    free(seen);
}

static void test_sorts(void)
{
    static const int64_t sizes[] = {0, 1, 2, 3, 31, 63, 64, 65, 127, 128, 1000, 4097, 20011};
    static const int32_t minruns[] = {0, 1, 2, 5, 16};
    for (size_t si = 0; si < sizeof sizes / sizeof *sizes; ++si) {
        const int64_t n = sizes[si];
        uint64_t* orig = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 1));
        uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 1));
        uint32_t* vals = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n + 1));
        int64_t* bounds = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 2));
        int64_t* log = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * (n + 1)));
        for (int kind = 0; kind < 5; ++kind) {
            fill(orig, n, kind);
            for (size_t mi = 0; mi < sizeof minruns / sizeof *minruns; ++mi) {
                for (int variant = 0; variant < 3 + 3; ++variant) {  /* 3..5: with ORC_DESC_RUNS */
                    memcpy(keys, orig, sizeof(uint64_t) * (size_t)n);
                    for (int64_t i = 0; i < n; ++i) vals[i] = (uint32_t)i;
                    orc_stats st;
                    const int v = variant < 3 ? variant : ((variant - 3) | ORC_DESC_RUNS);
                    int rc = orc_powersort(keys, vals, n, minruns[mi], v, &st, log, n);
                    CHECK(rc == 0, "powersort rc %d", rc);
                    check_stable(orig, keys, vals, n, "powersort");
                }
                /* the virtual-memory variant at small pages and at the page rule */
                static const int64_t pages[] = {0, 1, 2, 3, 7, 64};
                for (size_t pi = 0; pi < sizeof pages / sizeof *pages; ++pi)
                    for (int desc = 0; desc <= ORC_DESC_RUNS; desc += ORC_DESC_RUNS) {
                        memcpy(keys, orig, sizeof(uint64_t) * (size_t)n);
                        for (int64_t i = 0; i < n; ++i) vals[i] = (uint32_t)i;
                        orc_stats st;
                        orc_vm_stats vst;
                        const int rc = orc_vm_powersort(keys, pi % 2 ? vals : NULL, n, minruns[mi], pages[pi], desc,
                                                        &st, &vst, log, n);
                        CHECK(rc == 0, "vm powersort rc %d", rc);
                        if (pi % 2) check_stable(orig, keys, vals, n, "vm powersort");
                        for (int64_t i = 1; i < n; ++i) CHECK(keys[i - 1] <= keys[i], "vm keys out of order");
                        CHECK(st.mov_push + st.mov_merge + st.mov_copy <= st.merge_cost + 3 * n, "vm moves");
                    }
            }
            if (n < 2) continue;
            const int32_t ell = orc_minrun(n);
            uint8_t* dflag = (uint8_t*)malloc((size_t)(n + 1));
            const int64_t rd = orc_extract_runs_dir(orig, n, ell, 1, bounds, dflag);
            CHECK(rd >= 1 && bounds[0] == 0 && bounds[rd] == n, "extract_runs_dir bounds");
            free(dflag);
            const int64_t r = orc_extract_runs(orig, n, ell, bounds);
            CHECK(r >= 1 && bounds[0] == 0 && bounds[r] == n, "extract_runs bounds");
            uint8_t* powers = (uint8_t*)malloc((size_t)(r > 1 ? r - 1 : 1));
            orc_run_powers(bounds, r, n, powers);
            int64_t* nodes = (int64_t*)malloc(sizeof(int64_t) * (size_t)(4 * (r > 1 ? r - 1 : 1)));
            orc_tree_nodes(bounds, r, n, powers, nodes);
            int8_t* nbuf = (int8_t*)malloc((size_t)(r > 1 ? r - 1 : 1));
            int32_t* ndep = (int32_t*)malloc(sizeof(int32_t) * (size_t)(r > 1 ? r - 1 : 1));
            int64_t* segs = (int64_t*)malloc(sizeof(int64_t) * (size_t)(3 * r));
            int64_t mt = 0, mh = 0;
            const int64_t ns = orc_plan(bounds, r, n, powers, 64, nbuf, ndep, segs, &mt, &mh);
            CHECK(ns >= 1 && segs[0] == 0 && segs[3 * (ns - 1) + 1] == n, "plan covers the input");
            for (int64_t s = 1; s < ns; ++s) CHECK(segs[3 * s] == segs[3 * (s - 1) + 1], "plan segments contiguous");
            CHECK(mh <= mt, "M_hbm <= M");
            free(powers); free(nodes); free(nbuf); free(ndep); free(segs);
        }
        /* segmented: random cut points */
        if (n > 0) {
            fill(orig, n, 1);
            int64_t nseg = 1 + (int64_t)(next_rand() % 9);
            int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nseg + 1));
            off[0] = 0;
            off[nseg] = n;
            for (int64_t s = 1; s < nseg; ++s) off[s] = (int64_t)(next_rand() % (uint64_t)(n + 1));
            for (int64_t s = 1; s < nseg; ++s)  /* insertion sort of the cut points */
                for (int64_t t = s; t > 1 && off[t - 1] > off[t]; --t) { int64_t w = off[t]; off[t] = off[t - 1]; off[t - 1] = w; }
            memcpy(keys, orig, sizeof(uint64_t) * (size_t)n);
            for (int64_t i = 0; i < n; ++i) vals[i] = (uint32_t)i;
            CHECK(orc_segmented_powersort(keys, vals, off, nseg, 0, 1) == 0, "segmented rc");
            for (int64_t s = 0; s < nseg; ++s)
                for (int64_t i = off[s] + 1; i < off[s + 1]; ++i) {
                    CHECK(keys[i - 1] <= keys[i], "segment out of order");
                    if (keys[i - 1] == keys[i]) CHECK(vals[i - 1] < vals[i], "segment unstable");
                }
            free(off);
        }
        free(orig); free(keys); free(vals); free(bounds); free(log);
    }
}

static void test_merge(void)
{
    for (int trial = 0; trial < 50; ++trial) {
        const int64_t na = (int64_t)(next_rand() % 300), nb = (int64_t)(next_rand() % 300);
        uint64_t* a = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(na + 1));
        uint64_t* b = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
        uint32_t* va = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(na + 1));
        uint32_t* vb = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nb + 1));
        uint64_t* out = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(na + nb + 1));
        uint32_t* vo = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(na + nb + 1));
        uint64_t acc = 0;
        for (int64_t i = 0; i < na; ++i) { acc += next_rand() % 3; a[i] = acc; va[i] = (uint32_t)i; }
        acc = 0;
        for (int64_t i = 0; i < nb; ++i) { acc += next_rand() % 3; b[i] = acc; vb[i] = (uint32_t)(na + i); }
        orc_standard_merge(a, va, na, b, vb, nb, out, vo);
        for (int64_t i = 1; i < na + nb; ++i) {
            CHECK(out[i - 1] <= out[i], "merge out of order");
            if (out[i - 1] == out[i]) CHECK(vo[i - 1] < vo[i], "merge unstable");
        }
        free(a); free(b); free(va); free(vb); free(out); free(vo);
    }
}

static void test_learned(void)
{
    const int64_t n = 30000, m = 2048;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    fill(keys, n, 0);
    for (int64_t i = 0; i < n; ++i) keys[i] >>= (i % 40);  /* spread over bit lengths */
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    orc_sample_positions(n, m, 55, pos);
    uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)m);
    for (int64_t i = 0; i < m; ++i) { CHECK(pos[i] >= 0 && pos[i] < n, "sample position"); s[i] = keys[pos[i]]; }
    CHECK(orc_powersort(s, NULL, m, 0, 1, NULL, NULL, 0) == 0, "sample sort");
    const int32_t F = 20;
    const uint64_t z_lo = orc_feature(s[0], 64, F), z_hi = orc_feature(s[m - 1], 64, F);
    double* u = (double*)malloc(sizeof(double) * (size_t)m);
    for (int64_t i = 0; i < m; ++i)
        u[i] = z_hi > z_lo ? (double)(orc_feature(s[i], 64, F) - z_lo) / (double)(z_hi - z_lo) : 0.0;
    for (int32_t H = 1; H <= 64; H *= 4) {
        double* p = (double*)malloc(sizeof(double) * (size_t)(3 * H + 1));
        double* traj = (double*)malloc(sizeof(double) * (size_t)(3 * (3 * H + 1)));
        int32_t trained = -1;
        const double loss = orc_cdf_train2(u, m, H, 3, 64, 1e-3, p, &trained);
        CHECK(loss >= 0.0 && (trained == 0 || trained == 1), "train");
        orc_cdf_adam_steps(u, m, H, 3, 64, 1e-3, p, traj);
        uint64_t table[4097 + 1];
        int32_t sh = 0, kn = 0;
        orc_cdf_table(p, p + H, p + 2 * H, p[3 * H], H, z_lo, z_hi, 4096, table, &sh, &kn);
        CHECK(kn >= 1 && kn <= 4096, "knots");
        for (int32_t k = 1; k <= kn; ++k) CHECK(table[k - 1] <= table[k], "table monotone");
        const uint32_t B = 1024;
        uint64_t* ko = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
        int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (B + 1));
        orc_partition(keys, NULL, n, 64, F, z_lo, z_hi, table, sh, kn, B, ko, NULL, off);
        CHECK(off[0] == 0 && off[B] == n, "partition offsets");
        for (uint32_t b = 0; b < B; ++b) CHECK(off[b] <= off[b + 1], "offsets monotone");
        uint64_t mb = 0, sb = 0, dm[2], ds[2];
        orc_judge(s, m, 64, F, z_lo, z_hi, table, sh, kn, B, &mb, &sb, dm, ds);
        CHECK(mb < B, "judge bucket error");
        free(ko); free(off); free(p); free(traj);
    }
    free(keys); free(pos); free(s); free(u);
}

int main(void)
{
    test_sorts();
    test_merge();
    test_learned();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle self-test ok\n");
    return 0;
}

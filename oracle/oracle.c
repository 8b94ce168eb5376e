/*
 * Powersort CPU oracle: TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Everything here is the plain definition or the paper's algorithm in its
 * own order.  No blocking, no fusion, no parallelism.  Citations name the
 * paper's sections, algorithms and theorem.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* minrun rule (Section 5, "Algorithm variants"): start from l = n and  */
/* halve with rounding up until l < 64.                                */
/* ------------------------------------------------------------------ */
int32_t orc_minrun(int64_t n)
{
    int64_t l = n;
    while (l >= 64) l = (l + 1) / 2;
    return (int32_t)l;
}

/* ------------------------------------------------------------------ */
/* Power (theorem in Section 2): the least p such that some integer c   */
/* has (i+j)/(2n) < c / 2^p <= (j+k)/(2n).  Indices are 0-based and    */
/* half-open as in Algorithm 1's input[0,n).                           */
/* ------------------------------------------------------------------ */
int32_t orc_power_def(int64_t n, int64_t i, int64_t j, int64_t k)
{
    /* c exists iff floor((j+k) 2^p / 2n) > floor((i+j) 2^p / 2n). */
    for (int32_t p = 0; p < 127; ++p) {
        unsigned __int128 lo = ((unsigned __int128)(uint64_t)(i + j) << p) / (unsigned __int128)(2 * (uint64_t)n);
        unsigned __int128 hi = ((unsigned __int128)(uint64_t)(j + k) << p) / (unsigned __int128)(2 * (uint64_t)n);
        if (hi > lo) return p;
    }
    return -1;
}

/* Closed form of the same quantity (n <= 2^32): the first bit in which the
 * binary expansions of (i+j)/2n and (j+k)/2n differ.  A and B are those
 * expansions truncated to 32 bits. */
int32_t orc_power_closed(int64_t n, int64_t i, int64_t j, int64_t k)
{
    uint64_t A = ((uint64_t)(i + j) << 31) / (uint64_t)n;
    uint64_t B = ((uint64_t)(j + k) << 31) / (uint64_t)n;
    uint32_t x = (uint32_t)(A ^ B);
    int32_t lead = 0;
    while (lead < 32 && !(x & (0x80000000u >> lead))) ++lead;
    return lead + 1;
}

/* ------------------------------------------------------------------ */
/* ExtractRun (Section 2 and Section 3): a maximal non-decreasing run   */
/* starting at s, i.e. up to the first adjacent pair out of order;      */
/* only increasing runs are used (Section 5).                           */
/* ------------------------------------------------------------------ */
static int64_t natural_run_end(const uint64_t* x, int64_t s, int64_t n, int64_t* cmps)
{
    int64_t e = s + 1;
    while (e < n) {
        if (cmps) ++*cmps;
        if (x[e - 1] > x[e]) break;
        ++e;
    }
    return e;
}

/* With descending runs (Section 5 remark): when x[s+1] < x[s] the run is
 * the maximal strictly decreasing one from s (*desc = 1), else the maximal
 * non-decreasing one.  A strictly decreasing run has no equal keys, so
 * reversing it is its stable sort. */
static int64_t natural_run_end_dir(const uint64_t* x, int64_t s, int64_t n, int64_t* cmps, int* desc)
{
    *desc = 0;
    if (s + 1 >= n) return n;
    if (cmps) ++*cmps;
    if (x[s + 1] < x[s]) {
        int64_t e = s + 2;
        while (e < n) {
            if (cmps) ++*cmps;
            if (!(x[e] < x[e - 1])) break;
            ++e;
        }
        *desc = 1;
        return e;
    }
    return natural_run_end(x, s, n, cmps);
}

int64_t orc_extract_runs_dir(const uint64_t* x, int64_t n, int32_t minrun, int desc, int64_t* bounds,
                             uint8_t* desc_run)
{
    int64_t r = 0, s = 0;
    bounds[0] = 0;
    while (s < n) {
        int d = 0;
        int64_t e = desc ? natural_run_end_dir(x, s, n, NULL, &d) : natural_run_end(x, s, n, NULL);
        if (e - s < minrun) {
            e = (s + minrun < n) ? s + minrun : n;
            d = 0;
        }
        if (desc_run) desc_run[r] = (uint8_t)d;
        bounds[++r] = e;
        s = e;
    }
    return r;
}

int64_t orc_extract_runs(const uint64_t* x, int64_t n, int32_t minrun, int64_t* bounds)
{
    return orc_extract_runs_dir(x, n, minrun, 0, bounds, NULL);
}

/* Reverse x[s,e) (and v) in place. */
static void reverse_run(uint64_t* x, uint32_t* v, int64_t s, int64_t e, orc_stats* st)
{
    for (int64_t i = s, j = e - 1; i < j; ++i, --j) {
        uint64_t t = x[i]; x[i] = x[j]; x[j] = t;
        if (v) { uint32_t w = v[i]; v[i] = v[j]; v[j] = w; }
        st->mov_rev += 2;
    }
}

void orc_run_powers(const int64_t* bounds, int64_t r, int64_t n, uint8_t* powers)
{
    for (int64_t t = 0; t + 1 < r; ++t)
        powers[t] = (uint8_t)orc_power_def(n, bounds[t], bounds[t + 1], bounds[t + 2]);
}

/* Straight insertion sort of x[s,e) whose prefix x[s,sorted_end) is already
 * non-decreasing: this is how a short run is forced to length minrun. */
static void insertion_extend(uint64_t* x, uint32_t* v, int64_t s, int64_t sorted_end,
                             int64_t e, orc_stats* st)
{
    for (int64_t i = sorted_end; i < e; ++i) {
        uint64_t key = x[i];
        uint32_t val = v ? v[i] : 0;
        int64_t j = i;
        while (j > s) {
            st->cmp_ins++;
            if (!(x[j - 1] > key)) break;
            x[j] = x[j - 1];
            if (v) v[j] = v[j - 1];
            st->mov_ins++;
            --j;
        }
        if (j != i) {
            x[j] = key;
            if (v) v[j] = val;
            st->mov_ins++;
        }
    }
}

/* ExtractRun with the minrun extension: returns the run end.  With desc, a
 * strictly decreasing natural run is reversed first (also a short one,
 * before the insertion sort extends it). */
static int64_t extract_run(uint64_t* x, uint32_t* v, int64_t s, int64_t n, int32_t minrun, int desc,
                           orc_stats* st, double* H)
{
    int d = 0;
    int64_t e = desc ? natural_run_end_dir(x, s, n, &st->cmp_run, &d) : natural_run_end(x, s, n, &st->cmp_run);
    if (d) reverse_run(x, v, s, e, st);
    if (e - s < minrun) {
        int64_t forced = (s + minrun < n) ? s + minrun : n;
        insertion_extend(x, v, s, e, forced, st);
        e = forced;
    }
    st->runs++;
    double frac = (double)(e - s) / (double)n;
    *H += frac * log2(1.0 / frac);
    return e;
}

/* ------------------------------------------------------------------ */
/* StandardMerge (Algorithm 2, right): take from a iff a <= b, which    */
/* keeps equal keys in input order; the remainder is appended.          */
/* ------------------------------------------------------------------ */
void orc_standard_merge(const uint64_t* a, const uint32_t* va, int64_t na,
                        const uint64_t* b, const uint32_t* vb, int64_t nb,
                        uint64_t* out, uint32_t* vout)
{
    int64_t xa = 0, xb = 0, xr = 0;
    while (xa < na && xb < nb) {
        if (a[xa] <= b[xb]) { out[xr] = a[xa]; if (vout) vout[xr] = va[xa]; ++xa; }
        else                { out[xr] = b[xb]; if (vout) vout[xr] = vb[xb]; ++xb; }
        ++xr;
    }
    while (xa < na) { out[xr] = a[xa]; if (vout) vout[xr] = va[xa]; ++xa; ++xr; }
    while (xb < nb) { out[xr] = b[xb]; if (vout) vout[xr] = vb[xb]; ++xb; ++xr; }
}

/* Pingpong MergeBuffers (Section 3): a = stackBuf[i,j), b = input[j,k),
 * output input[i,k) written left to right.  Unread b never gets overwritten
 * because the write index never passes the read index of b. */
static void merge_lr_into_input(uint64_t* A, uint32_t* VA, const uint64_t* B, const uint32_t* VB,
                                int64_t i, int64_t j, int64_t k, orc_stats* st)
{
    int64_t xa = i, xb = j, xr = i;
    while (xa < j && xb < k) {
        st->cmp_merge++;
        if (B[xa] <= A[xb]) { A[xr] = B[xa]; if (VA) VA[xr] = VB[xa]; ++xa; }
        else                { A[xr] = A[xb]; if (VA) VA[xr] = VA[xb]; ++xb; }
        ++xr; st->mov_merge++;
    }
    while (xa < j) { A[xr] = B[xa]; if (VA) VA[xr] = VB[xa]; ++xa; ++xr; st->mov_merge++; }
    /* a remainder of b already sits at its final place */
}

/* The "last pop" merge of Section 3: a = stackBuf[i,j), b = input[j,k),
 * output stackBuf[i,k) written right to left.  Stable: on ties the element
 * of b is emitted first when going right to left. */
static void merge_rl_into_stack(const uint64_t* A, const uint32_t* VA, uint64_t* B, uint32_t* VB,
                                int64_t i, int64_t j, int64_t k, orc_stats* st)
{
    int64_t ya = j, yb = k, yr = k;
    while (ya > i && yb > j) {
        st->cmp_merge++;
        --yr;
        if (B[ya - 1] > A[yb - 1]) { B[yr] = B[ya - 1]; if (VB) VB[yr] = VB[ya - 1]; --ya; }
        else                       { B[yr] = A[yb - 1]; if (VB) VB[yr] = VA[yb - 1]; --yb; }
        st->mov_merge++;
    }
    while (yb > j) { --yr; B[yr] = A[yb - 1]; if (VB) VB[yr] = VA[yb - 1]; --yb; st->mov_merge++; }
    /* a remainder of a already sits at its final place */
}

/* CPython-style MergeBuffers (Section 2): copy the smaller run to aux and
 * merge back into input[i,k). */
static void merge_cpython(uint64_t* A, uint32_t* VA, uint64_t* aux, uint32_t* vaux,
                          int64_t i, int64_t j, int64_t k, orc_stats* st)
{
    if (j - i <= k - j) {
        for (int64_t t = i; t < j; ++t) { aux[t - i] = A[t]; if (VA) vaux[t - i] = VA[t]; st->mov_merge++; }
        int64_t xa = 0, na = j - i, xb = j, xr = i;
        while (xa < na && xb < k) {
            st->cmp_merge++;
            if (aux[xa] <= A[xb]) { A[xr] = aux[xa]; if (VA) VA[xr] = vaux[xa]; ++xa; }
            else                  { A[xr] = A[xb];  if (VA) VA[xr] = VA[xb];  ++xb; }
            ++xr; st->mov_merge++;
        }
        while (xa < na) { A[xr] = aux[xa]; if (VA) VA[xr] = vaux[xa]; ++xa; ++xr; st->mov_merge++; }
    } else {
        for (int64_t t = j; t < k; ++t) { aux[t - j] = A[t]; if (VA) vaux[t - j] = VA[t]; st->mov_merge++; }
        int64_t ya = j, yb = k - j, yr = k;
        while (ya > i && yb > 0) {
            st->cmp_merge++;
            --yr;
            if (A[ya - 1] > aux[yb - 1]) { A[yr] = A[ya - 1]; if (VA) VA[yr] = VA[ya - 1]; --ya; }
            else                         { A[yr] = aux[yb - 1]; if (VA) VA[yr] = vaux[yb - 1]; --yb; }
            st->mov_merge++;
        }
        while (yb > 0) { --yr; A[yr] = aux[yb - 1]; if (VA) VA[yr] = vaux[yb - 1]; --yb; st->mov_merge++; }
    }
}

typedef struct { int64_t lo, hi; int32_t power; } stack_entry;

/* ------------------------------------------------------------------ */
/* Algorithm 1 ("Abstract Powersort") with one of the buffer schemes.   */
/* The final collapse pops the stack at each step.                      */
/* ------------------------------------------------------------------ */
int orc_powersort(uint64_t* keys, uint32_t* vals, int64_t n, int32_t minrun,
                  int variant, orc_stats* st_out, int64_t* merge_log, int64_t log_cap)
{
    orc_stats st;
    memset(&st, 0, sizeof st);
    st.n = n;
    const int desc = (variant & ORC_DESC_RUNS) != 0;
    variant &= ~ORC_DESC_RUNS;
    if (n < 0 || variant < 0 || variant > 2) return -1;
    if (n <= 1) {
        if (n == 1) st.runs = 1;
        if (st_out) *st_out = st;
        return 0;
    }
    int32_t l = minrun > 0 ? minrun : orc_minrun(n);
    int64_t buf_len = (variant == ORC_CPYTHON) ? n / 2 + 1 : n;
    uint64_t* B = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)buf_len);
    uint32_t* VB = vals ? (uint32_t*)malloc(sizeof(uint32_t) * (size_t)buf_len) : NULL;
    stack_entry* stack = (stack_entry*)malloc(sizeof(stack_entry) * 130);
    if (!B || (vals && !VB) || !stack) { free(B); free(VB); free(stack); return -1; }
    int64_t height = 0, nlog = 0;
    double H = 0.0;

#define LOG_MERGE(I, J, K)                                                    \
    do {                                                                      \
        st.merges++;                                                          \
        st.merge_cost += (K) - (I);                                           \
        if (merge_log && nlog < log_cap) {                                    \
            merge_log[3 * nlog] = (I); merge_log[3 * nlog + 1] = (J);         \
            merge_log[3 * nlog + 2] = (K);                                    \
        }                                                                     \
        ++nlog;                                                               \
    } while (0)

    int64_t c_lo = 0;
    int64_t c_hi = extract_run(keys, vals, 0, n, l, desc, &st, &H);
    int curr_in_stackbuf = 0; /* Pingpong: where curr currently lives */
    while (c_hi < n) {
        int64_t nx_hi = extract_run(keys, vals, c_hi, n, l, desc, &st, &H);
        int32_t p = orc_power_def(n, c_lo, c_hi, nx_hi);
        while (height > 0 && stack[height - 1].power >= p) {
            stack_entry top = stack[height - 1];
            int last = (height == 1) || (stack[height - 2].power < p);
            LOG_MERGE(top.lo, c_lo, c_hi);
            if (variant == ORC_CPYTHON) {
                merge_cpython(keys, vals, B, VB, top.lo, c_lo, c_hi, &st);
            } else if (variant == ORC_PINGPONG_LASTPOP && last) {
                merge_rl_into_stack(keys, vals, B, VB, top.lo, c_lo, c_hi, &st);
                curr_in_stackbuf = 1;
            } else {
                merge_lr_into_input(keys, vals, B, VB, top.lo, c_lo, c_hi, &st);
                curr_in_stackbuf = 0;
            }
            c_lo = top.lo;
            --height;
        }
        if (variant != ORC_CPYTHON && !curr_in_stackbuf) {
            /* Push copies curr into stackBuf (at most once per element). */
            for (int64_t t = c_lo; t < c_hi; ++t) {
                B[t] = keys[t];
                if (vals) VB[t] = vals[t];
                st.mov_push++;
            }
        }
        stack[height].lo = c_lo; stack[height].hi = c_hi; stack[height].power = p;
        ++height;
        if (height > st.max_stack) st.max_stack = height;
        c_lo = c_hi; c_hi = nx_hi; curr_in_stackbuf = 0;
    }
    while (height > 0) {
        stack_entry top = stack[height - 1];
        LOG_MERGE(top.lo, c_lo, c_hi);
        if (variant == ORC_CPYTHON) merge_cpython(keys, vals, B, VB, top.lo, c_lo, c_hi, &st);
        else merge_lr_into_input(keys, vals, B, VB, top.lo, c_lo, c_hi, &st);
        c_lo = top.lo;
        --height;
    }
#undef LOG_MERGE
    st.entropy = H;
    if (st_out) *st_out = st;
    free(B); free(VB); free(stack);
    return 0;
}

int orc_segmented_powersort(uint64_t* keys, uint32_t* vals, const int64_t* seg_off,
                            int64_t nseg, int32_t minrun, int variant)
{
    for (int64_t s = 0; s < nseg; ++s) {
        int64_t a = seg_off[s], b = seg_off[s + 1];
        if (b < a) return -1;
        if (orc_powersort(keys + a, vals ? vals + a : NULL, b - a, minrun, variant, NULL, NULL, 0))
            return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Tree form of Algorithm 1's merges: boundary t merges its left and    */
/* right neighbourhoods up to the nearest boundary of smaller power.    */
/* ------------------------------------------------------------------ */
static int64_t nearest_smaller_left(const uint8_t* P, int64_t t)
{
    for (int64_t u = t - 1; u >= 0; --u) if (P[u] < P[t]) return u;
    return -1;
}

static int64_t nearest_smaller_right(const uint8_t* P, int64_t nb, int64_t t)
{
    for (int64_t u = t + 1; u < nb; ++u) if (P[u] < P[t]) return u;
    return -1;
}

void orc_tree_nodes(const int64_t* bounds, int64_t r, int64_t n,
                    const uint8_t* powers, int64_t* nodes)
{
    int64_t nb = r - 1;
    for (int64_t t = 0; t < nb; ++t) {
        int64_t lu = nearest_smaller_left(powers, t);
        int64_t ru = nearest_smaller_right(powers, nb, t);
        nodes[4 * t + 0] = lu >= 0 ? bounds[lu + 1] : 0;
        nodes[4 * t + 1] = bounds[t + 1];
        nodes[4 * t + 2] = ru >= 0 ? bounds[ru + 1] : n;
        nodes[4 * t + 3] = powers[t];
    }
}

/* Pingpong placement (Section 3 read as a tree): the root writes to the
 * input A; every node writes to the buffer opposite its parent, so both
 * children of a node sit in one buffer and the node writes to the other. */
int64_t orc_plan(const int64_t* bounds, int64_t r, int64_t n, const uint8_t* powers,
                 int64_t T, int8_t* node_buf, int32_t* node_depth, int64_t* segs,
                 int64_t* m_total, int64_t* m_hbm)
{
    int64_t nb = r > 0 ? r - 1 : 0;
    int64_t* parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb + 1));
    int64_t* L = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb + 1));
    int64_t* R = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb + 1));
    int64_t mt = 0, mh = 0, ns = 0;
    for (int64_t t = 0; t < nb; ++t) {
        int64_t lu = nearest_smaller_left(powers, t);
        int64_t ru = nearest_smaller_right(powers, nb, t);
        L[t] = lu >= 0 ? bounds[lu + 1] : 0;
        R[t] = ru >= 0 ? bounds[ru + 1] : n;
        if (lu < 0) parent[t] = ru;
        else if (ru < 0) parent[t] = lu;
        else parent[t] = powers[lu] > powers[ru] ? lu : ru;
        mt += R[t] - L[t];
        if (R[t] - L[t] > T) mh += R[t] - L[t];
    }
    /* depth by walking to the root (plain, quadratic in the worst case) */
    for (int64_t t = 0; t < nb; ++t) {
        int32_t d = 0;
        for (int64_t u = parent[t]; u >= 0; u = parent[u]) ++d;
        node_depth[t] = d;
        node_buf[t] = (int8_t)(d & 1);
    }
    /* segments: cut at the positions of nodes longer than T */
    int64_t prev_pos = 0, prev_b = -1;
    for (int64_t t = 0; t <= nb; ++t) {
        int is_cut = (t < nb) && (R[t] - L[t] > T);
        if (t < nb && !is_cut) continue;
        int64_t pos = (t < nb) ? bounds[t + 1] : n;
        /* parent of segment [prev_pos,pos): the adjacent long node with the
         * larger power (the deeper one), or the root position if none. */
        int64_t par;
        if (prev_b < 0 && t == nb) par = -1;
        else if (prev_b < 0) par = t;
        else if (t == nb) par = prev_b;
        else par = powers[prev_b] > powers[t] ? prev_b : t;
        int8_t buf = par < 0 ? 0 : (int8_t)((node_depth[par] + 1) & 1);
        segs[3 * ns + 0] = prev_pos;
        segs[3 * ns + 1] = pos;
        segs[3 * ns + 2] = buf;
        ++ns;
        prev_pos = pos;
        prev_b = t;
    }
    if (m_total) *m_total = mt;
    if (m_hbm) *m_hbm = mh;
    free(parent); free(L); free(R);
    return ns;
}

/* ------------------------------------------------------------------ */
/* Learned CDF partitioner, fp64 reference.                             */
/* ------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea, Flood 2014; Vigna's public-domain version). */
uint64_t orc_splitmix64(uint64_t* state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Output number `counter` (0-based) of a SplitMix64 stream seeded with seed. */
uint64_t orc_mix64(uint64_t seed, uint64_t counter)
{
    uint64_t s = seed + counter * 0x9E3779B97F4A7C15ull; /* state after `counter` steps */
    return orc_splitmix64(&s);
}

void orc_sample_positions(int64_t n, int64_t m, uint64_t seed, int64_t* pos)
{
    uint64_t s = seed;
    for (int64_t i = 0; i < m; ++i) pos[i] = (int64_t)(orc_splitmix64(&s) % (uint64_t)n);
}

/* Monotone integer feature: bit length of the key, then the next fbits
 * bits below its leading one. */
uint64_t orc_feature(uint64_t key, int32_t key_bits, int32_t fbits)
{
    if (key_bits == 32) key &= 0xFFFFFFFFull;
    int32_t b = 0;
    for (uint64_t t = key; t; t >>= 1) ++b;
    if (b == 0) return 0;
    uint64_t mask = (fbits >= 64) ? ~0ull : ((1ull << fbits) - 1);
    uint64_t rest = key & ((b - 1 >= 64) ? ~0ull : ((1ull << (b - 1)) - 1)); /* drop the leading one */
    uint64_t mant;
    if (b - 1 >= fbits) mant = rest >> (b - 1 - fbits);
    else mant = rest << (fbits - (b - 1));
    return ((uint64_t)b << fbits) | (mant & mask);
}

static double relu(double a) { return a > 0.0 ? a : 0.0; }

double orc_mlp_forward(const double* w1, const double* b1, const double* w2, double b2,
                       int32_t H, double u)
{
    double f = b2;
    for (int32_t h = 0; h < H; ++h) f += w2[h] * relu(w1[h] * u + b1[h]);
    return f;
}

/* Mean squared error over a minibatch and its gradient (backpropagation
 * through one hidden ReLU layer).  Returns the loss. */
double orc_mlp_grad(const double* w1, const double* b1, const double* w2, double b2,
                    int32_t H, const double* u, const double* y, int64_t nb,
                    double* g_w1, double* g_b1, double* g_w2, double* g_b2)
{
    for (int32_t h = 0; h < H; ++h) { g_w1[h] = 0; g_b1[h] = 0; g_w2[h] = 0; }
    *g_b2 = 0;
    double loss = 0.0;
    for (int64_t i = 0; i < nb; ++i) {
        double f = orc_mlp_forward(w1, b1, w2, b2, H, u[i]);
        double err = f - y[i];
        loss += err * err;
        double dfd = 2.0 * err / (double)nb;
        *g_b2 += dfd;
        for (int32_t h = 0; h < H; ++h) {
            double a = w1[h] * u[i] + b1[h];
            if (a > 0.0) {
                g_w2[h] += dfd * a;
                g_w1[h] += dfd * w2[h] * u[i];
                g_b1[h] += dfd * w2[h];
            }
        }
    }
    return loss / (double)nb;
}

/* Knot spacing of the table: segments of 2^shift feature units, the least
 * power of two that covers [z_lo, z_hi] with at most K segments. */
void orc_cdf_grid(uint64_t z_lo, uint64_t z_hi, int32_t K, int32_t* shift, int32_t* knots)
{
    uint64_t range = z_hi > z_lo ? z_hi - z_lo : 0;
    int32_t sh = 0;
    while (((range + (1ull << sh) - 1) >> sh) > (uint64_t)K) ++sh;
    uint64_t kk = (range + (1ull << sh) - 1) >> sh;
    *shift = sh;
    *knots = kk > 0 ? (int32_t)kk : 1;
}

/* Compile the model into knots+1 monotone fixed-point positions (Q32 of
 * [0,1]) at feature offsets s * 2^shift. */
void orc_cdf_table(const double* w1, const double* b1, const double* w2, double b2,
                   int32_t H, uint64_t z_lo, uint64_t z_hi, int32_t K, uint64_t* table,
                   int32_t* shift_out, int32_t* knots_out)
{
    int32_t sh, kn;
    orc_cdf_grid(z_lo, z_hi, K, &sh, &kn);
    uint64_t range = z_hi > z_lo ? z_hi - z_lo : 0;
    uint64_t run_max = 0;
    for (int32_t s = 0; s <= kn; ++s) {
        double u = range ? (double)((uint64_t)s << sh) / (double)range : 0.0;
        if (u > 1.0) u = 1.0;
        double v = orc_mlp_forward(w1, b1, w2, b2, H, u);
        if (!(v > 0.0)) v = 0.0;
        if (v > 1.0) v = 1.0;
        double q = floor(v * 4294967296.0);
        uint64_t qi = q >= 4294967295.0 ? 4294967295ull : (uint64_t)q;
        if (qi < run_max) qi = run_max;
        run_max = qi;
        table[s] = qi;
    }
    *shift_out = sh;
    *knots_out = kn;
}

/* Position of a key under the compiled model, F(key) in Q32: linear
 * interpolation between the table's knots in the feature coordinate, all in
 * integers. */
uint64_t orc_cdf_pos(uint64_t key, int32_t key_bits, int32_t fbits, uint64_t z_lo, uint64_t z_hi,
                     const uint64_t* table, int32_t shift, int32_t knots)
{
    uint64_t z = orc_feature(key, key_bits, fbits);
    uint64_t range = z_hi > z_lo ? z_hi - z_lo : 0;
    uint64_t d = z <= z_lo ? 0 : (z - z_lo > range ? range : z - z_lo);
    uint64_t seg = d >> shift;
    if (seg >= (uint64_t)knots) return table[knots];
    uint64_t rem = d & ((1ull << shift) - 1);
    return table[seg] + (((table[seg + 1] - table[seg]) * rem) >> shift);
}

/* Bucket of a key: its position scaled to B buckets. */
uint32_t orc_bucket_of(uint64_t key, int32_t key_bits, int32_t fbits, uint64_t z_lo,
                       uint64_t z_hi, const uint64_t* table, int32_t shift, int32_t knots,
                       uint32_t B)
{
    uint64_t pos = orc_cdf_pos(key, key_bits, fbits, z_lo, z_hi, table, shift, knots);
    uint64_t b = (pos * (uint64_t)B) >> 32;
    return (uint32_t)(b >= B ? B - 1 : b);
}

/* Error judge of the compiled model on the sorted sample x_0 <= ... <=
 * x_{m-1}, whose targets are y_i = (i + 1/2) / m.  Per sample point:
 *   bucket error  |bucket(x_i) - floor(B y_i)|              (integer)
 *   CDF error     |B F(x_i) - B y_i| = B d_i / (2^33 m),
 *                 d_i = |2m pos_i - 2^32 (2i + 1)|           (exact, 128-bit)
 * Returns the maximum and the sum of both over the sample (the 128-bit
 * values as low/high words). */
void orc_judge(const uint64_t* sorted, int64_t m, int32_t key_bits, int32_t fbits, uint64_t z_lo,
               uint64_t z_hi, const uint64_t* table, int32_t shift, int32_t knots, uint32_t B,
               uint64_t* max_bucket_err, uint64_t* sum_bucket_err, uint64_t d_max[2], uint64_t d_sum[2])
{
    uint64_t mb = 0, sb = 0;
    unsigned __int128 dm = 0, ds = 0;
    for (int64_t i = 0; i < m; ++i) {
        uint64_t pos = orc_cdf_pos(sorted[i], key_bits, fbits, z_lo, z_hi, table, shift, knots);
        uint64_t b = (pos * (uint64_t)B) >> 32;
        if (b >= B) b = B - 1;
        uint64_t want = ((uint64_t)B * (uint64_t)(2 * i + 1)) / (uint64_t)(2 * m);
        uint64_t eb = b > want ? b - want : want - b;
        if (eb > mb) mb = eb;
        sb += eb;
        unsigned __int128 a = (unsigned __int128)pos * (unsigned __int128)(2 * m);
        unsigned __int128 t = (unsigned __int128)(2 * i + 1) << 32;
        unsigned __int128 d = a > t ? a - t : t - a;
        if (d > dm) dm = d;
        ds += d;
    }
    *max_bucket_err = mb;
    *sum_bucket_err = sb;
    d_max[0] = (uint64_t)dm; d_max[1] = (uint64_t)(dm >> 64);
    d_sum[0] = (uint64_t)ds; d_sum[1] = (uint64_t)(ds >> 64);
}

/* Stable counting sort by bucket id: the plain definition of the partition. */
void orc_partition(const uint64_t* keys, const uint32_t* vals, int64_t n,
                   int32_t key_bits, int32_t fbits, uint64_t z_lo, uint64_t z_hi,
                   const uint64_t* table, int32_t shift, int32_t knots, uint32_t B,
                   uint64_t* keys_out, uint32_t* vals_out, int64_t* offsets)
{
    uint32_t* id = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    for (uint32_t b = 0; b <= B; ++b) offsets[b] = 0;
    for (int64_t i = 0; i < n; ++i) {
        id[i] = orc_bucket_of(keys[i], key_bits, fbits, z_lo, z_hi, table, shift, knots, B);
        offsets[id[i] + 1]++;
    }
    for (uint32_t b = 0; b < B; ++b) offsets[b + 1] += offsets[b];
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)B);
    for (uint32_t b = 0; b < B; ++b) cur[b] = offsets[b];
    for (int64_t i = 0; i < n; ++i) {
        int64_t dst = cur[id[i]]++;
        keys_out[dst] = keys[i];
        if (vals && vals_out) vals_out[dst] = vals[i];
    }
    free(cur);
    free(id);
}

/* Model initialisation from the sorted sample: H hinges at evenly spaced
 * sample quantiles, output weights chosen so the model interpolates the
 * empirical CDF (i+1/2)/m linearly between the hinges. */
void orc_cdf_init(const double* u, int64_t m, int32_t H, double* w1, double* b1,
                  double* w2, double* b2)
{
    double* q = (double*)malloc(sizeof(double) * (size_t)H);
    double* y = (double*)malloc(sizeof(double) * (size_t)H);
    double* slope = (double*)malloc(sizeof(double) * (size_t)H);
    for (int32_t h = 0; h < H; ++h) {
        int64_t qi = (H > 1) ? ((int64_t)h * (m - 1)) / (H - 1) : 0;
        q[h] = u[qi];
        y[h] = ((double)qi + 0.5) / (double)m;
        if (h > 0 && q[h] <= q[h - 1]) q[h] = q[h - 1] + ORC_KNOT_GAP;
    }
    for (int32_t h = 0; h + 1 < H; ++h) slope[h] = (y[h + 1] - y[h]) / (q[h + 1] - q[h]);
    for (int32_t h = 0; h < H; ++h) {
        w1[h] = 1.0;
        b1[h] = -q[h];
        double right = (h + 1 < H) ? slope[h] : 0.0;
        double left = (h > 0) ? slope[h - 1] : 0.0;
        w2[h] = right - left;
    }
    *b2 = y[0];
    free(q); free(y); free(slope);
}

/* Adam (Kingma and Ba 2015) with bias correction; step counts from 1. */
void orc_adam_update(double* p, const double* g, double* m1, double* m2, int32_t n,
                     int64_t step, double lr)
{
    double c1 = 1.0 - pow(ORC_BETA1, (double)step);
    double c2 = 1.0 - pow(ORC_BETA2, (double)step);
    for (int32_t i = 0; i < n; ++i) {
        m1[i] = ORC_BETA1 * m1[i] + (1.0 - ORC_BETA1) * g[i];
        m2[i] = ORC_BETA2 * m2[i] + (1.0 - ORC_BETA2) * g[i] * g[i];
        p[i] -= lr * (m1[i] / c1) / (sqrt(m2[i] / c2) + ORC_ADAM_EPS);
    }
}

/* Mean squared error of the model over every `stride`-th sample point. */
double orc_cdf_loss(const double* w1, const double* b1, const double* w2, double b2, int32_t H,
                    const double* u, int64_t m, int64_t stride)
{
    double s = 0.0;
    int64_t c = 0;
    for (int64_t i = 0; i < m; i += stride) {
        double e = orc_mlp_forward(w1, b1, w2, b2, H, u[i]) - ((double)i + 0.5) / (double)m;
        s += e * e;
        ++c;
    }
    return c ? s / (double)c : 0.0;
}

/* Adam steps on minibatches, from the parameters the caller passes in:
 * minibatch j of step s (both 0-based) is the sample point at index
 * (s*nb + j) * ORC_BATCH_STRIDE mod m with target (index + 1/2)/m, the
 * gradient is the minibatch MSE's (orc_mlp_grad), and the Adam step count
 * starts at 1.  params = [w1(H) b1(H) w2(H) b2] is updated in place; traj
 * (nullable) receives the parameters after every step, steps x (3H+1). */
void orc_cdf_adam_steps(const double* u, int64_t m, int32_t H, int32_t steps, int32_t nb,
                        double lr, double* params, double* traj)
{
    int32_t np_ = 3 * H + 1;
    double* p = params;
    double* g = (double*)calloc((size_t)np_, sizeof(double));
    double* m1 = (double*)calloc((size_t)np_, sizeof(double));
    double* m2 = (double*)calloc((size_t)np_, sizeof(double));
    double* ub = (double*)malloc(sizeof(double) * (size_t)nb);
    double* yb = (double*)malloc(sizeof(double) * (size_t)nb);
    for (int32_t s = 0; s < steps; ++s) {
        for (int32_t j = 0; j < nb; ++j) {
            uint64_t idx = (((uint64_t)s * (uint64_t)nb + (uint64_t)j) * ORC_BATCH_STRIDE) % (uint64_t)m;
            ub[j] = u[idx];
            yb[j] = ((double)idx + 0.5) / (double)m;
        }
        orc_mlp_grad(p, p + H, p + 2 * H, p[3 * H], H, ub, yb, nb, g, g + H, g + 2 * H, g + 3 * H);
        orc_adam_update(p, g, m1, m2, np_, s + 1, lr);
        if (traj) memcpy(traj + (size_t)s * (size_t)np_, p, sizeof(double) * (size_t)np_);
    }
    free(g); free(m1); free(m2); free(ub); free(yb);
}

/* Full training: quantile initialisation, `steps` Adam steps
 * (orc_cdf_adam_steps), then the trained model is kept when its strided
 * loss is at most the initial model's, else the initial model is restored.
 * params = [w1(H) b1(H) w2(H) b2].  Returns the final strided loss;
 * *trained (nullable) is 1 when the trained model was kept. */
double orc_cdf_train2(const double* u, int64_t m, int32_t H, int32_t steps, int32_t nb,
                      double lr, double* params, int32_t* trained)
{
    int32_t np_ = 3 * H + 1;
    double* p = params;
    double* init = (double*)malloc(sizeof(double) * (size_t)np_);
    orc_cdf_init(u, m, H, p, p + H, p + 2 * H, p + 3 * H);
    double loss0 = orc_cdf_loss(p, p + H, p + 2 * H, p[3 * H], H, u, m, ORC_LOSS_STRIDE);
    memcpy(init, p, sizeof(double) * (size_t)np_);
    orc_cdf_adam_steps(u, m, H, steps, nb, lr, p, NULL);
    double loss1 = orc_cdf_loss(p, p + H, p + 2 * H, p[3 * H], H, u, m, ORC_LOSS_STRIDE);
    int32_t keep = loss1 <= loss0;
    if (!keep) { memcpy(p, init, sizeof(double) * (size_t)np_); loss1 = loss0; }
    if (trained) *trained = keep;
    free(init);
    return loss1;
}

double orc_cdf_train(const double* u, int64_t m, int32_t H, int32_t steps, int32_t nb,
                     double lr, double* params)
{
    return orc_cdf_train2(u, m, H, steps, nb, lr, params, NULL);
}

/* ------------------------------------------------------------------ */
/* Virtual-Memory Powersort (Section 4).                                */
/* Memory is cut into pages of P elements: the input array's pages and  */
/* extra pages appended on demand.  A buffer is a list of pages whose   */
/* concatenation, from an offset into its first page, holds its         */
/* elements in order; every page but the first and the last is full.   */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t* pages;  /* physical page ids */
    int64_t npages, cap;
    int64_t head;    /* offset of the first element inside pages[0] */
    int64_t len;     /* elements */
} vm_buffer;

typedef struct {
    uint64_t* key;     /* memory: input pages first, then extra pages */
    uint32_t* val;     /* NULL when sorting keys only */
    int64_t P, n;
    int64_t input_pages, npages_total, cap_pages;
    int64_t* free_list;
    int64_t nfree, free_cap;
    int64_t live_meta, live_buffers;
    orc_stats* st;
    orc_vm_stats* vst;
    int failed;
} vm_mem;

static int64_t vm_log2_ceil(int64_t n)
{
    int64_t l = 0;
    while (((int64_t)1 << l) < n) ++l;
    return l;
}

int64_t orc_vm_page(int64_t n, int32_t rec_words)
{
    if (n < 2) return 1;
    const double t = rec_words > 0 ? (double)rec_words : 1.0;
    const double target = sqrt((double)n / (t * (double)vm_log2_ceil(n)));
    int64_t p = 1;
    while ((double)(2 * p) <= target) p *= 2;
    return p;
}

static void vm_note_meta(vm_mem* m)
{
    const int64_t words = m->live_meta + m->nfree;
    if (words > m->vst->meta_words) m->vst->meta_words = words;
    if (m->live_buffers > m->vst->max_buffers) m->vst->max_buffers = m->live_buffers;
    const int64_t extra = m->npages_total - m->input_pages;
    if (extra > m->vst->extra_pages) m->vst->extra_pages = extra;
}

static int64_t vm_new_page(vm_mem* m)
{
    if (m->nfree > 0) return m->free_list[--m->nfree];
    if (m->npages_total == m->cap_pages) {
        /* grow the memory by whole pages (the extra pages of Section 4) */
        int64_t cap = m->cap_pages * 2 + 4;
        uint64_t* k = (uint64_t*)realloc(m->key, sizeof(uint64_t) * (size_t)(cap * m->P));
        if (!k) { m->failed = 1; return 0; }
        m->key = k;
        if (m->val) {
            uint32_t* v = (uint32_t*)realloc(m->val, sizeof(uint32_t) * (size_t)(cap * m->P));
            if (!v) { m->failed = 1; return 0; }
            m->val = v;
        }
        m->cap_pages = cap;
    }
    const int64_t p = m->npages_total++;
    vm_note_meta(m);
    return p;
}

static void vm_free_page(vm_mem* m, int64_t p)
{
    /* the input's last page, when partial, is never handed out again */
    if (p == m->input_pages - 1 && m->n % m->P) return;
    if (m->nfree == m->free_cap) {
        m->free_cap = m->free_cap * 2 + 16;
        int64_t* f = (int64_t*)realloc(m->free_list, sizeof(int64_t) * (size_t)m->free_cap);
        if (!f) { m->failed = 1; return; }
        m->free_list = f;
    }
    m->free_list[m->nfree++] = p;
    vm_note_meta(m);
}

static void vm_buf_init(vm_mem* m, vm_buffer* b)
{
    b->pages = NULL; b->npages = 0; b->cap = 0; b->head = 0; b->len = 0;
    m->live_buffers++;
    vm_note_meta(m);
}

static void vm_buf_add_page(vm_mem* m, vm_buffer* b, int64_t p)
{
    if (b->npages == b->cap) {
        b->cap = b->cap * 2 + 4;
        int64_t* q = (int64_t*)realloc(b->pages, sizeof(int64_t) * (size_t)b->cap);
        if (!q) { m->failed = 1; return; }
        b->pages = q;
    }
    b->pages[b->npages++] = p;
    m->live_meta++;
    vm_note_meta(m);
}

static void vm_buf_done(vm_mem* m, vm_buffer* b)
{
    m->live_meta -= b->npages;
    m->live_buffers--;
    free(b->pages);
    b->pages = NULL; b->npages = 0; b->cap = 0; b->len = 0; b->head = 0;
}

/* PushBack: one element into the buffer's last page (a new page when it is
 * full). */
static void vm_push_back(vm_mem* m, vm_buffer* b, uint64_t k, uint32_t v)
{
    const int64_t pos = b->head + b->len;
    if (pos == b->npages * m->P) vm_buf_add_page(m, b, vm_new_page(m));
    if (m->failed) return;
    const int64_t at = b->pages[pos / m->P] * m->P + pos % m->P;
    m->key[at] = k;
    if (m->val) m->val[at] = v;
    b->len++;
}

/* PopFront: drop the first element; a page left empty goes to the free list. */
static void vm_pop_front(vm_mem* m, vm_buffer* b)
{
    b->head++;
    b->len--;
    if (b->head == m->P || b->len == 0) {
        /* the page leaves the buffer's list before it joins the free list */
        const int64_t p = b->pages[0];
        memmove(b->pages, b->pages + 1, sizeof(int64_t) * (size_t)(b->npages - 1));
        b->npages--;
        m->live_meta--;
        b->head = 0;
        vm_free_page(m, p);
        if (b->len == 0) {
            /* an emptied buffer gives back every page it still holds */
            const int64_t k = b->npages;
            m->live_meta -= k;
            b->npages = 0;
            for (int64_t i = 0; i < k; ++i) vm_free_page(m, b->pages[i]);
        }
    }
}

static inline uint64_t vm_front_key(const vm_mem* m, const vm_buffer* b)
{
    return m->key[b->pages[0] * m->P + b->head];
}

static inline uint32_t vm_front_val(const vm_mem* m, const vm_buffer* b)
{
    return m->val ? m->val[b->pages[0] * m->P + b->head] : 0u;
}

/* MergeRuns page by page: StandardMerge's rule (ties to a), consuming a and
 * b from the front and appending to r (PageMerge of Algorithm 2 in its
 * simplest form: one element per step, page ends handled by the buffer
 * operations). */
static void vm_merge(vm_mem* m, vm_buffer* a, vm_buffer* b, vm_buffer* r)
{
    while (a->len > 0 && b->len > 0 && !m->failed) {
        m->st->cmp_merge++;
        if (vm_front_key(m, a) <= vm_front_key(m, b)) {
            vm_push_back(m, r, vm_front_key(m, a), vm_front_val(m, a));
            vm_pop_front(m, a);
        } else {
            vm_push_back(m, r, vm_front_key(m, b), vm_front_val(m, b));
            vm_pop_front(m, b);
        }
        m->st->mov_merge++;
    }
    while (a->len > 0 && !m->failed) {
        vm_push_back(m, r, vm_front_key(m, a), vm_front_val(m, a));
        vm_pop_front(m, a);
        m->st->mov_merge++;
    }
    while (b->len > 0 && !m->failed) {
        vm_push_back(m, r, vm_front_key(m, b), vm_front_val(m, b));
        vm_pop_front(m, b);
        m->st->mov_merge++;
    }
}

/* Copy (Section 4): the final buffer r (head 0) into the input array, page
 * by page: when input page t is still in use by r at another position, its
 * contents move to a new page first; then r's page t moves into place.  A
 * page that receives its final contents leaves the free list (linear scan,
 * as the paper allows), so no later step hands it out again. */
static void vm_copy_out(vm_mem* m, vm_buffer* r)
{
    const int64_t P = m->P, n = m->n;
    for (int64_t t = 0; t < r->npages && !m->failed; ++t) {
        for (int64_t f = 0; f < m->nfree; ++f)
            if (m->free_list[f] == t) { m->free_list[f] = m->free_list[--m->nfree]; break; }
        if (r->pages[t] == t) continue;
        for (int64_t j = t + 1; j < r->npages; ++j) {
            if (r->pages[j] != t) continue;
            const int64_t q = vm_new_page(m);
            if (m->failed) return;
            const int64_t cnt = (j + 1) * P <= n ? P : n - j * P;
            for (int64_t i = 0; i < cnt; ++i) {
                m->key[q * P + i] = m->key[t * P + i];
                if (m->val) m->val[q * P + i] = m->val[t * P + i];
                m->st->mov_copy++;
            }
            r->pages[j] = q;
            break;
        }
        const int64_t src = r->pages[t];
        const int64_t cnt = (t + 1) * P <= n ? P : n - t * P;
        for (int64_t i = 0; i < cnt; ++i) {
            m->key[t * P + i] = m->key[src * P + i];
            if (m->val) m->val[t * P + i] = m->val[src * P + i];
            m->st->mov_copy++;
        }
        r->pages[t] = t;
        vm_free_page(m, src);
    }
}

int orc_vm_powersort(uint64_t* keys, uint32_t* vals, int64_t n, int32_t minrun, int64_t page, int desc,
                     orc_stats* st_out, orc_vm_stats* vst_out, int64_t* merge_log, int64_t log_cap)
{
    orc_stats st;
    orc_vm_stats vst;
    memset(&st, 0, sizeof st);
    memset(&vst, 0, sizeof vst);
    st.n = n;
    if (n < 0) return -1;
    const int64_t P = page > 0 ? page : orc_vm_page(n, vals ? 2 : 1);
    vst.page = P;
    if (n <= 1) {
        if (n == 1) st.runs = 1;
        if (st_out) *st_out = st;
        if (vst_out) *vst_out = vst;
        return 0;
    }
    int32_t l = minrun > 0 ? minrun : orc_minrun(n);
    vm_mem m;
    memset(&m, 0, sizeof m);
    m.P = P; m.n = n; m.st = &st; m.vst = &vst;
    m.input_pages = (n + P - 1) / P;
    m.npages_total = m.input_pages;
    m.cap_pages = m.input_pages + 4;
    vst.input_pages = m.input_pages;
    m.key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m.cap_pages * P));
    m.val = vals ? (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(m.cap_pages * P)) : NULL;
    vm_buffer* stack = (vm_buffer*)malloc(sizeof(vm_buffer) * 130);
    int32_t* spow = (int32_t*)malloc(sizeof(int32_t) * 130);
    int64_t* slo = (int64_t*)malloc(sizeof(int64_t) * 130);
    if (!m.key || (vals && !m.val) || !stack || !spow || !slo) {
        free(m.key); free(m.val); free(stack); free(spow); free(slo);
        return -1;
    }
    memcpy(m.key, keys, sizeof(uint64_t) * (size_t)n);
    if (vals) memcpy(m.val, vals, sizeof(uint32_t) * (size_t)n);
    /* work: the input's pages, consumed from the front */
    vm_buffer work;
    vm_buf_init(&m, &work);
    for (int64_t p = 0; p < m.input_pages; ++p) vm_buf_add_page(&m, &work, p);
    work.len = n;
    int64_t height = 0, nlog = 0, s = 0;
    double H = 0.0;

#define VM_LOG(I, J, K)                                                       \
    do {                                                                      \
        st.merges++;                                                          \
        st.merge_cost += (K) - (I);                                           \
        if (merge_log && nlog < log_cap) {                                    \
            merge_log[3 * nlog] = (I); merge_log[3 * nlog + 1] = (J);         \
            merge_log[3 * nlog + 2] = (K);                                    \
        }                                                                     \
        ++nlog;                                                               \
    } while (0)

    /* ExtractRun: the run [s, e) is formed where it lies in the input (the
     * insertion sort of a forced run and the reversal of a decreasing one
     * act there, on elements work still owns), then moved into a buffer of
     * its own by PushBack / PopFront */
    vm_buffer curr, next;
    int64_t c_lo = 0, c_hi = 0;
#define VM_EXTRACT(BUF, LO, HI)                                                         \
    do {                                                                                \
        (LO) = s;                                                                       \
        (HI) = extract_run(m.key, m.val, s, n, l, desc, &st, &H);                       \
        vm_buf_init(&m, &(BUF));                                                        \
        for (int64_t i = s; i < (HI) && !m.failed; ++i) {                               \
            vm_push_back(&m, &(BUF), vm_front_key(&m, &work), vm_front_val(&m, &work)); \
            vm_pop_front(&m, &work);                                                    \
            st.mov_push++;                                                              \
        }                                                                               \
        s = (HI);                                                                       \
    } while (0)

    VM_EXTRACT(curr, c_lo, c_hi);
    while (c_hi < n && !m.failed) {
        int64_t nx_lo = 0, nx_hi = 0;
        VM_EXTRACT(next, nx_lo, nx_hi);
        int32_t p = orc_power_def(n, c_lo, c_hi, nx_hi);
        while (height > 0 && spow[height - 1] >= p && !m.failed) {
            vm_buffer r;
            vm_buf_init(&m, &r);
            VM_LOG(slo[height - 1], c_lo, c_hi);
            vm_merge(&m, &stack[height - 1], &curr, &r);
            vm_buf_done(&m, &stack[height - 1]);
            vm_buf_done(&m, &curr);
            curr = r;
            c_lo = slo[height - 1];
            --height;
        }
        stack[height] = curr; spow[height] = p; slo[height] = c_lo;
        ++height;
        if (height > st.max_stack) st.max_stack = height;
        curr = next; c_lo = nx_lo; c_hi = nx_hi;
    }
    while (height > 0 && !m.failed) {
        vm_buffer r;
        vm_buf_init(&m, &r);
        VM_LOG(slo[height - 1], c_lo, c_hi);
        vm_merge(&m, &stack[height - 1], &curr, &r);
        vm_buf_done(&m, &stack[height - 1]);
        vm_buf_done(&m, &curr);
        curr = r;
        c_lo = slo[height - 1];
        --height;
    }
#undef VM_EXTRACT
#undef VM_LOG
    if (!m.failed) vm_copy_out(&m, &curr);
    vm_buf_done(&m, &curr);
    vm_buf_done(&m, &work);
    const int failed = m.failed;
    if (!failed) {
        memcpy(keys, m.key, sizeof(uint64_t) * (size_t)n);
        if (vals) memcpy(vals, m.val, sizeof(uint32_t) * (size_t)n);
    }
    st.entropy = H;
    if (st_out) *st_out = st;
    if (vst_out) *vst_out = vst;
    free(m.key); free(m.val); free(m.free_list); free(stack); free(spow); free(slo);
    return failed ? -1 : 0;
}

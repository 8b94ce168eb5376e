/*
 * Powersort CPU oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of what the GPU sort
 * computes, written from the paper "Virtual-Memory Powersort" (Algorithm 1
 * "Abstract Powersort", the Power theorem of Section 2, Pingpong Powersort in
 * Section 3, StandardMerge in Algorithm 2, the minrun rule of Section 5).
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * may load this library.  The product path never calls it and shares no code
 * with it.
 *
 * Keys are unsigned 64-bit here; 32-bit keys are widened by the caller, which
 * preserves their unsigned order.  Values are 32-bit payloads that move with
 * their keys (NULL = keys only).
 */
#ifndef VMPS_ORACLE_H
#define VMPS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n;           /* input length                                  */
    int64_t runs;        /* r: runs after minrun extension                */
    int64_t merges;      /* number of MergeBuffers calls                  */
    int64_t merge_cost;  /* M: sum of merge input lengths (Def. merge cost) */
    int64_t max_stack;   /* largest run-stack height seen                 */
    int64_t cmp_run;     /* comparisons spent on run detection            */
    int64_t cmp_ins;     /* comparisons spent inside insertion sort       */
    int64_t cmp_merge;   /* comparisons spent inside merges               */
    int64_t mov_ins;     /* element writes by insertion sort              */
    int64_t mov_push;    /* element copies input -> stack buffer          */
    int64_t mov_merge;   /* element writes by merges (incl. aux copies)   */
    double  entropy;     /* run-length entropy H over the extended runs   */
    int64_t mov_rev;     /* element writes by descending-run reversals    */
    int64_t mov_copy;    /* element writes by the final Copy (VM variant) */
} orc_stats;

/* Memory of the virtual-memory variant (Section 4). */
typedef struct {
    int64_t page;          /* P: elements per page                           */
    int64_t input_pages;   /* pages the input array is cut into              */
    int64_t extra_pages;   /* most pages beyond the input's in use at once   */
    int64_t meta_words;    /* most page-list and free-list entries at once   */
    int64_t max_buffers;   /* most live buffers (stack + curr + next + merge) */
} orc_vm_stats;

/* Variants of Algorithm 1 the oracle can run. */
enum {
    ORC_PINGPONG = 0,          /* Section 3: stack runs in stackBuf, curr in input   */
    ORC_PINGPONG_LASTPOP = 1,  /* Section 3 + right-to-left last pop into stackBuf   */
    ORC_CPYTHON = 2,           /* Section 2: copy smaller run to aux, merge back     */
    /* flag, or-ed into any variant: ExtractRun also takes maximal strictly
     * decreasing runs and reverses them (the remark on decreasing runs in
     * Section 5); strictness keeps equal keys in input order */
    ORC_DESC_RUNS = 4
};

int32_t orc_minrun(int64_t n);
int32_t orc_power_def(int64_t n, int64_t i, int64_t j, int64_t k);
int32_t orc_power_closed(int64_t n, int64_t i, int64_t j, int64_t k);

/* Sequential ExtractRun chain over x[0,n) (no sorting). bounds gets r+1
 * entries (bounds[0]=0, bounds[r]=n); returns r. */
int64_t orc_extract_runs(const uint64_t* x, int64_t n, int32_t minrun, int64_t* bounds);

/* The same chain with descending runs (ORC_DESC_RUNS) when desc != 0; desc_run
 * (nullable, r entries) gets 1 for every run that is a maximal strictly
 * decreasing run of at least minrun elements (reversed by the sort). */
int64_t orc_extract_runs_dir(const uint64_t* x, int64_t n, int32_t minrun, int desc, int64_t* bounds,
                             uint8_t* desc_run);

/* Power of every run boundary: powers[t] for runs t,t+1 (t < r-1). */
void orc_run_powers(const int64_t* bounds, int64_t r, int64_t n, uint8_t* powers);

/* Algorithm 1 on keys[0,n) (+vals). minrun<=0 means the Section 5 rule.
 * merge_log (nullable) receives (i,j,k) triples in execution order.
 * Returns 0 on success, -1 on allocation failure or bad arguments. */
int orc_powersort(uint64_t* keys, uint32_t* vals, int64_t n, int32_t minrun,
                  int variant, orc_stats* st, int64_t* merge_log, int64_t log_cap);

/* Virtual-Memory Powersort (Section 4): Algorithm 1 with every buffer a list
 * of pages of `page` elements taken from a free list (consumed pages of the
 * input and of merged runs go back to it; an empty free list allocates an
 * extra page), merges page by page (PageMerge of Algorithm 2), and a final
 * Copy that permutes pages into the input array.  page <= 0: the rule of
 * orc_vm_page.  desc: ORC_DESC_RUNS or 0.  Counters as orc_powersort
 * (mov_push: run extraction into pages, mov_copy: the final Copy).
 * Returns 0, or -1 on bad arguments / allocation failure. */
int orc_vm_powersort(uint64_t* keys, uint32_t* vals, int64_t n, int32_t minrun, int64_t page, int desc,
                     orc_stats* st, orc_vm_stats* vst, int64_t* merge_log, int64_t log_cap);

/* Page size of Section 4: about sqrt(n / (T log2 n)) elements for records of
 * T words, rounded down to a power of two (at least 1). */
int64_t orc_vm_page(int64_t n, int32_t rec_words);

/* Same, over independent segments seg_off[0..nseg] of one array; every
 * segment is an instance of its own (minrun <= 0: the rule for its length). */
int orc_segmented_powersort(uint64_t* keys, uint32_t* vals, const int64_t* seg_off,
                            int64_t nseg, int32_t minrun, int variant);

/* StandardMerge (Algorithm 2, right) with the remainder appended. */
void orc_standard_merge(const uint64_t* a, const uint32_t* va, int64_t na,
                        const uint64_t* b, const uint32_t* vb, int64_t nb,
                        uint64_t* out, uint32_t* vout);

/* Tree form of the merge schedule: for boundary t, node (L, mid, R, power)
 * where L/R are the nearest boundaries with smaller power (else 0 / n).
 * nodes gets 4*(r-1) int64 values. */
void orc_tree_nodes(const int64_t* bounds, int64_t r, int64_t n,
                    const uint8_t* powers, int64_t* nodes);

/* Pingpong placement of the tree with an LDS tile of T elements.
 *   node_buf[t]  : buffer (0 = input A, 1 = workspace B) node t writes to
 *   node_depth[t]: depth of node t in the merge tree (root = 0)
 *   segs         : the maximal subtrees of size <= T (or single runs longer
 *                  than T) as (start, end, buffer) triples, in order;
 *                  returns their count.
 *   m_total / m_hbm: merge cost M and the part of it in nodes longer than T. */
int64_t orc_plan(const int64_t* bounds, int64_t r, int64_t n, const uint8_t* powers,
                 int64_t T, int8_t* node_buf, int32_t* node_depth, int64_t* segs,
                 int64_t* m_total, int64_t* m_hbm);

/* ---- learned CDF partitioner (fp64 reference) ---- */
#define ORC_KNOT_GAP     1e-6                 /* separation of coincident knots */
#define ORC_BETA1        0.9
#define ORC_BETA2        0.999
#define ORC_ADAM_EPS     1e-8
#define ORC_BATCH_STRIDE 0x9E3779B1ull        /* odd: visits every sample mod 2^k */
#define ORC_LOSS_STRIDE  64
uint64_t orc_splitmix64(uint64_t* state);
uint64_t orc_mix64(uint64_t seed, uint64_t counter);
void     orc_sample_positions(int64_t n, int64_t m, uint64_t seed, int64_t* pos);
uint64_t orc_feature(uint64_t key, int32_t key_bits, int32_t fbits);
double   orc_mlp_forward(const double* w1, const double* b1, const double* w2, double b2,
                         int32_t H, double u);
double   orc_mlp_grad(const double* w1, const double* b1, const double* w2, double b2,
                      int32_t H, const double* u, const double* y, int64_t nb,
                      double* g_w1, double* g_b1, double* g_w2, double* g_b2);
void     orc_cdf_grid(uint64_t z_lo, uint64_t z_hi, int32_t K, int32_t* shift, int32_t* knots);
void     orc_cdf_table(const double* w1, const double* b1, const double* w2, double b2,
                       int32_t H, uint64_t z_lo, uint64_t z_hi, int32_t K, uint64_t* table,
                       int32_t* shift, int32_t* knots);
uint64_t orc_cdf_pos(uint64_t key, int32_t key_bits, int32_t fbits, uint64_t z_lo, uint64_t z_hi,
                     const uint64_t* table, int32_t shift, int32_t knots);
uint32_t orc_bucket_of(uint64_t key, int32_t key_bits, int32_t fbits, uint64_t z_lo,
                       uint64_t z_hi, const uint64_t* table, int32_t shift, int32_t knots,
                       uint32_t B);
void     orc_cdf_init(const double* u, int64_t m, int32_t H, double* w1, double* b1,
                      double* w2, double* b2);
void     orc_adam_update(double* p, const double* g, double* m1, double* m2, int32_t n,
                         int64_t step, double lr);
double   orc_cdf_loss(const double* w1, const double* b1, const double* w2, double b2, int32_t H,
                      const double* u, int64_t m, int64_t stride);
/* Adam steps from caller parameters, no initialisation, no model choice. */
void     orc_cdf_adam_steps(const double* u, int64_t m, int32_t H, int32_t steps, int32_t nb,
                            double lr, double* params, double* traj);
double   orc_cdf_train(const double* u, int64_t m, int32_t H, int32_t steps, int32_t nb,
                       double lr, double* params);
double   orc_cdf_train2(const double* u, int64_t m, int32_t H, int32_t steps, int32_t nb,
                        double lr, double* params, int32_t* trained);
void     orc_partition(const uint64_t* keys, const uint32_t* vals, int64_t n,
                       int32_t key_bits, int32_t fbits, uint64_t z_lo, uint64_t z_hi,
                       const uint64_t* table, int32_t shift, int32_t knots, uint32_t B,
                       uint64_t* keys_out, uint32_t* vals_out, int64_t* offsets);
void     orc_judge(const uint64_t* sorted, int64_t m, int32_t key_bits, int32_t fbits,
                   uint64_t z_lo, uint64_t z_hi, const uint64_t* table, int32_t shift,
                   int32_t knots, uint32_t B, uint64_t* max_bucket_err, uint64_t* sum_bucket_err,
                   uint64_t d_max[2], uint64_t d_sum[2]);

#ifdef __cplusplus
}
#endif
#endif

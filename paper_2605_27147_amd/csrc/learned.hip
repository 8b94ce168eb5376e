// Learned CDF partitioning in front of Powersort.
//
// sample -> sort the sample (the plain Powersort path) -> features ->
// train (forward/backward/Adam in one workgroup) -> compile to an integer
// knot table -> stable two-level scatter by bucket id -> Powersort of every
// bucket as an instance of its own (the segmented path).  Buckets are
// increasing key ranges and the scatter is stable, so the output is the
// stable sort for any model; the model only decides how even the buckets
// are, and buckets longer than the LDS tile fall back to the merge levels.
#include <string.h>

#include <type_traits>

#include "vmps_internal.hpp"

namespace vmps {

constexpr uint32_t PART_TILE = 8192;  // keys per histogram / scatter workgroup
constexpr int PART_NT = 512;
constexpr int PART_NW = PART_NT / 64;
constexpr int PART_RND = PART_TILE / PART_NT;  // keys per thread
constexpr int PART_DMAX = 512;                  // digits of a scatter level (9 bits)
constexpr uint64_t BATCH_STRIDE = 0x9E3779B1ull;  // odd: visits every sample mod 2^k
constexpr int LOSS_STRIDE = 64;
constexpr float KNOT_GAP = 1e-6f;

// ------------------------------------------------------------ helpers --
// Output `counter` (0-based) of SplitMix64 seeded with `seed`.
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Monotone feature: bit length, then the fbits bits below the leading one.
__device__ inline uint64_t feature_of(uint64_t key, int fbits)
{
    if (!key) return 0;
    const int b = 64 - __clzll((long long)key);
    const uint64_t rest = key & ((1ull << (b - 1)) - 1);
    const uint64_t mant = (b - 1 >= fbits) ? (rest >> (b - 1 - fbits)) : (rest << (fbits - (b - 1)));
    return ((uint64_t)b << fbits) | (mant & ((1ull << fbits) - 1));
}

struct ModelArgs {
    uint64_t z_lo, range;
    int fbits, shift, knots;
    uint32_t B;
    const uint64_t* table;
};

// F(key) of the compiled table in Q32: integer interpolation between knots.
__device__ inline uint64_t cdf_pos(uint64_t key, const ModelArgs& M)
{
    const uint64_t z = feature_of(key, M.fbits);
    const uint64_t d = z <= M.z_lo ? 0 : (z - M.z_lo > M.range ? M.range : z - M.z_lo);
    const uint64_t seg = d >> M.shift;
    if (seg >= (uint64_t)M.knots) return M.table[M.knots];
    const uint64_t t0 = M.table[seg], t1 = M.table[seg + 1];
    return t0 + (((t1 - t0) * (d & ((1ull << M.shift) - 1))) >> M.shift);
}

__device__ inline uint32_t bucket_of(uint64_t key, const ModelArgs& M)
{
    const uint64_t b = (cdf_pos(key, M) * M.B) >> 32;
    return (uint32_t)(b >= M.B ? M.B - 1 : b);
}

// The same bucket in 32-bit arithmetic, for a monotone table whose values
// fit 32 bits (every compiled table).  The feature is below 2^31 (bit length
// at most 64, at most 24 fraction bits), so z_lo and the range clamped to
// 2^31 - 1 give the same d; (t1 - t0) times the offset inside the segment is
// below 2^63 and its quotient by 2^shift below t1 - t0, so every
// intermediate of cdf_pos is reproduced exactly.
struct ModelArgs32 {
    uint32_t z_lo, range, fbits, shift, seg_shift, frac_mask, knots, B;
    const uint32_t* table;  // knots + 1 entries
};

__device__ inline ModelArgs32 model_args32(const ModelArgs& M, const uint32_t* table32)
{
    ModelArgs32 a;
    a.z_lo = M.z_lo > 0x7fffffffull ? 0x7fffffffu : (uint32_t)M.z_lo;
    a.range = M.range > 0x7fffffffull ? 0x7fffffffu : (uint32_t)M.range;
    a.fbits = (uint32_t)M.fbits;
    a.shift = (uint32_t)M.shift;
    a.seg_shift = M.shift < 32 ? (uint32_t)M.shift : 31u;  // d < 2^31: a shift of 31 already gives 0
    a.frac_mask = M.shift < 32 ? (1u << M.shift) - 1u : 0xffffffffu;
    a.knots = (uint32_t)M.knots;
    a.B = M.B;
    a.table = table32;
    return a;
}

__device__ inline uint32_t bucket_of32(uint64_t key, const ModelArgs32& M)
{
    // feature: bit length b, then the fbits bits below the leading one
    const uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)key;
    const uint32_t c = hi ? (uint32_t)__clz(hi) : 32u + (uint32_t)__clz(lo);  // 64 for key 0
    const uint32_t top = (uint32_t)((key << (c & 63)) >> 32);  // leading one at bit 31
    const uint32_t mant = (top >> (31u - M.fbits)) & ((1u << M.fbits) - 1u);
    const uint32_t z = key ? ((64u - c) << M.fbits) | mant : 0u;
    const uint32_t d = z <= M.z_lo ? 0u : min(z - M.z_lo, M.range);
    const uint32_t seg = d >> M.seg_shift;
    const uint32_t sc = seg < M.knots ? seg : M.knots - 1u;
    const uint32_t t0 = M.table[sc], t1 = M.table[sc + 1];
    const uint64_t prod = (uint64_t)(t1 - t0) * (uint64_t)(d & M.frac_mask);
    const uint32_t pos = seg < M.knots ? t0 + (uint32_t)(prod >> M.shift) : M.table[M.knots];
    const uint32_t b = __umulhi(pos, M.B);
    return b >= M.B ? M.B - 1u : b;
}

// Bucket arguments of a compiled model (uniform loads at kernel start).
__device__ inline ModelArgs model_args(const vmps_cdf_model* model, uint32_t B)
{
    ModelArgs a;
    a.z_lo = model->z_lo;
    a.range = model->z_hi > model->z_lo ? model->z_hi - model->z_lo : 0;
    // a caller-built model is clamped to the table it can hold
    a.fbits = min(max(model->feature_bits, 1), 24);
    a.shift = min(max(model->shift, 0), 62);
    a.knots = min(max(model->knots, 1), VMPS_CDF_MAX_KNOTS);
    a.B = B;
    a.table = model->table;
    return a;
}

// ------------------------------------------------------------ sample --
template <typename K>
__global__ void k_sample_gather(const K* __restrict__ keys, uint64_t n, uint64_t m, uint64_t seed,
                                K* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    out[i] = keys[splitmix64_at(seed, i) % n];
}

template <typename K>
__global__ void k_cdf_features(const K* __restrict__ s, uint64_t m, int key_bits, int fbits,
                               float* __restrict__ u, vmps_cdf_model* model)
{
    const uint64_t z_lo = feature_of((uint64_t)s[0], fbits), z_hi = feature_of((uint64_t)s[m - 1], fbits);
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        model->z_lo = z_lo;
        model->z_hi = z_hi;
        model->key_bits = key_bits;
        model->feature_bits = fbits;
    }
    if (i >= m) return;
    const uint64_t range = z_hi - z_lo;
    u[i] = range ? (float)(feature_of((uint64_t)s[i], fbits) - z_lo) / (float)range : 0.f;
}

// ------------------------------------------------------------- model --
// v of another lane by a DPP lane pattern (VALU only, no LDS traffic).
template <int CTRL>
__device__ inline float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over the H lanes of a lane group (H divides 64), the xor butterfly
// order: lane ^ 1 and lane ^ 2 by quad permutations; then, with every quad
// (and later every 8 lanes) holding one common value, the mirror inside 8
// and inside 16 lanes reads the same values as lane ^ 4 and lane ^ 8; lane
// ^ 16 by a swizzle inside 32 lanes, lane ^ 32 by a shuffle.
template <int H>
__device__ inline float group_sum(float v)
{
    static_assert(H >= 2 && H <= 64 && (H & (H - 1)) == 0, "lane group of a power of two");
    v += dpp_f32<0xB1>(v);                 // quad_perm [1,0,3,2]
    if (H > 2) v += dpp_f32<0x4E>(v);      // quad_perm [2,3,0,1]
    if (H > 4) v += dpp_f32<0x141>(v);     // row_half_mirror
    if (H > 8) v += dpp_f32<0x140>(v);     // row_mirror
    if (H > 16) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));  // xor 16
    if (H > 32) v += __shfl_xor(v, 32, 64);
    return v;
}

constexpr int TRAIN_NT = 1024;  // one-workgroup kernels (initialisation, loss, compile)
constexpr int STEP_NT = 256;    // workgroups of one Adam step
constexpr int STEP_PTS = 256;   // minibatch points per step workgroup
constexpr int NP_PAD = 3 * VMPS_CDF_MAX_HIDDEN + 64;  // parameter slots, padded

template <int NT>
struct TrainLds {
    float p[3 * VMPS_CDF_MAX_HIDDEN + 1];
    float g[3 * VMPS_CDF_MAX_HIDDEN + 1];
    float m1[3 * VMPS_CDF_MAX_HIDDEN + 1];
    float m2[3 * VMPS_CDF_MAX_HIDDEN + 1];
    float best[3 * VMPS_CDF_MAX_HIDDEN + 1];
    float pw1[NT], pb1[NT], pw2[NT];
    float pb2[NT], pl[NT];
    float q[VMPS_CDF_MAX_HIDDEN], y[VMPS_CDF_MAX_HIDDEN];
    float bu[NT], by[NT];  // minibatch points, staged per chunk
    float loss;
};

// Gradient of the squared error summed over `cnt` points, each term scaled
// by `inv` (2/nb for the mean over a minibatch of nb points): forward pass,
// then backpropagation through the hidden ReLU layer.  The points are
// staged in LDS, NT at a time.  Thread t owns hidden unit t % H of lane
// group t / H; groups take the staged points in turn; partial sums are
// reduced in a fixed order, so the result does not depend on timing.
// point(j, u, y) yields point j.  Writes S.g and S.loss (the sum of the
// squared errors divided by cnt).
template <int H, int NT, typename Point>
__device__ void batch_grad(TrainLds<NT>& S, int cnt_all, float inv, Point point)
{
    constexpr int G = NT / H;
    const int t = threadIdx.x, h = t % H, grp = t / H;
    const float w1 = S.p[h], b1 = S.p[H + h], w2 = S.p[2 * H + h], b2 = S.p[3 * H];
    float aw1 = 0.f, ab1 = 0.f, aw2 = 0.f, ab2 = 0.f, al = 0.f;
    for (int base = 0; base < cnt_all; base += NT) {
        const int cnt = cnt_all - base < NT ? cnt_all - base : NT;
        if (t < cnt) {
            float uu, yy;
            point(base + t, uu, yy);
            S.bu[t] = uu;
            S.by[t] = yy;
        }
        __syncthreads();
        // UB points at a time: their cross-lane sums are independent, so the
        // shuffles overlap; the accumulation below keeps the point order
        constexpr int UB = 8;
        int j = grp;
        for (; j + (UB - 1) * G < cnt; j += UB * G) {
            float uu[UB], yy[UB], aa[UB], rr[UB], ff[UB];
#pragma unroll
            for (int q = 0; q < UB; ++q) {
                uu[q] = S.bu[j + q * G];
                yy[q] = S.by[j + q * G];
                aa[q] = w1 * uu[q] + b1;
                rr[q] = aa[q] > 0.f ? aa[q] : 0.f;
                ff[q] = w2 * rr[q];
            }
#pragma unroll
            for (int q = 0; q < UB; ++q) ff[q] = group_sum<H>(ff[q]);
#pragma unroll
            for (int q = 0; q < UB; ++q) {
                const float e = (ff[q] + b2) - yy[q];
                const float dfd = inv * e;
                if (aa[q] > 0.f) {
                    aw2 += dfd * rr[q];
                    aw1 += dfd * w2 * uu[q];
                    ab1 += dfd * w2;
                }
                ab2 += dfd;
                al += e * e;
            }
        }
        for (; j < cnt; j += G) {
            const float u = S.bu[j], y = S.by[j];
            const float a = w1 * u + b1;
            const float r = a > 0.f ? a : 0.f;
            const float f = group_sum<H>(w2 * r) + b2;
            const float e = f - y;
            const float dfd = inv * e;
            if (a > 0.f) {
                aw2 += dfd * r;
                aw1 += dfd * w2 * u;
                ab1 += dfd * w2;
            }
            ab2 += dfd;
            al += e * e;
        }
        __syncthreads();
    }
    S.pw1[t] = aw1; S.pb1[t] = ab1; S.pw2[t] = aw2;
    if (h == 0) { S.pb2[grp] = ab2; S.pl[grp] = al; }
    __syncthreads();
    if (t < H) {
        float s1 = 0.f, s2 = 0.f, s3 = 0.f;
        for (int gg = 0; gg < G; ++gg) {
            s1 += S.pw1[gg * H + t];
            s2 += S.pb1[gg * H + t];
            s3 += S.pw2[gg * H + t];
        }
        S.g[t] = s1; S.g[H + t] = s2; S.g[2 * H + t] = s3;
    } else if (t == H) {
        float s = 0.f, l = 0.f;
        for (int gg = 0; gg < G; ++gg) { s += S.pb2[gg]; l += S.pl[gg]; }
        S.g[3 * H] = s;
        S.loss = cnt_all > 0 ? l / (float)cnt_all : 0.f;
    }
    __syncthreads();
}

template <int H>
__global__ __launch_bounds__(TRAIN_NT) void k_cdf_grad(const float* __restrict__ params, const float* __restrict__ u,
                                                       const float* __restrict__ y, int nb, float* __restrict__ grad,
                                                       float* __restrict__ loss)
{
    __shared__ TrainLds<TRAIN_NT> S;
    const int t = threadIdx.x;
    if (t < 3 * H + 1) S.p[t] = params[t];
    __syncthreads();
    batch_grad<H, TRAIN_NT>(S, nb, 2.f / (float)nb, [&](int j, float& uu, float& yy) { uu = u[j]; yy = y[j]; });
    if (t < 3 * H + 1) grad[t] = S.g[t];
    if (t == 0) *loss = S.loss;
}

template <int H>
__device__ float model_eval(const float* p, float u)
{
    float f = p[3 * H];
#pragma unroll 8
    for (int h = 0; h < H; ++h) {
        const float a = p[h] * u + p[H + h];
        f += p[2 * H + h] * (a > 0.f ? a : 0.f);
    }
    return f;
}

// Compile the parameters in p into the model's knot table (block-wide).
template <int H>
__device__ void compile_table(const float* p, vmps_cdf_model* model, uint64_t z_lo, uint64_t z_hi, int K,
                              uint32_t* scan_lds)
{
    const int t = threadIdx.x;
    const uint64_t range = z_hi > z_lo ? z_hi - z_lo : 0;
    int sh = 0;
    while (((range + (1ull << sh) - 1) >> sh) > (uint64_t)K) ++sh;
    uint64_t kk = (range + (1ull << sh) - 1) >> sh;
    const int kn = kk > 0 ? (int)kk : 1;
    // knots, then a running maximum (block scan of per-thread maxima)
    constexpr int PER = (VMPS_CDF_MAX_KNOTS + 1 + TRAIN_NT - 1) / TRAIN_NT;
    uint32_t v[PER];
    uint32_t mx = 0;
    for (int j = 0; j < PER; ++j) {
        const int s = t * PER + j;
        uint32_t q = 0;
        if (s <= kn) {
            float u = range ? (float)((uint64_t)s << sh) / (float)range : 0.f;
            if (u > 1.f) u = 1.f;
            float f = model_eval<H>(p, u);
            if (!(f > 0.f)) f = 0.f;
            if (f > 1.f) f = 1.f;
            const float qf = floorf(f * 4294967296.0f);
            q = qf >= 4294967295.0f ? 4294967295u : (uint32_t)qf;
        }
        mx = max(mx, q);
        v[j] = mx;
    }
    scan_lds[t] = mx;
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (int k = 0; k < TRAIN_NT; ++k) { uint32_t x = scan_lds[k]; scan_lds[k] = run; run = max(run, x); }
    }
    __syncthreads();
    const uint32_t before = scan_lds[t];
    for (int j = 0; j < PER; ++j) {
        const int s = t * PER + j;
        if (s <= kn) model->table[s] = (uint64_t)max(before, v[j]);
    }
    if (t == 0) {
        model->knots = kn;
        model->shift = sh;
        model->hidden = H;
    }
    if (t < H) {
        model->w1[t] = p[t];
        model->b1[t] = p[H + t];
        model->w2[t] = p[2 * H + t];
    }
    if (t == 0) model->b2 = p[3 * H];
    __syncthreads();
}

template <int H>
__global__ __launch_bounds__(TRAIN_NT) void k_cdf_compile(const float* __restrict__ params, uint64_t z_lo,
                                                          uint64_t z_hi, int key_bits, int fbits, int K,
                                                          vmps_cdf_model* model)
{
    __shared__ float p[3 * VMPS_CDF_MAX_HIDDEN + 1];
    __shared__ uint32_t scan_lds[TRAIN_NT];
    const int t = threadIdx.x;
    if (t < 3 * H + 1) p[t] = params[t];
    if (t == 0) {
        model->z_lo = z_lo; model->z_hi = z_hi; model->key_bits = key_bits; model->feature_bits = fbits;
        model->trained = 0; model->loss_init = 0.f; model->loss_final = 0.f;
    }
    __syncthreads();
    compile_table<H>(p, model, z_lo, z_hi, K, scan_lds);
}

// Training runs as a chain of launches on the caller's stream: k_cdf_init
// (one workgroup: the quantile initialisation), k_cdf_step for s = 0 ..
// steps (Adam step s, then the gradient of minibatch s spread over
// workgroups; the first and the last launch also split the strided loss of
// their parameters over workgroups), k_cdf_finish (one workgroup: the choice
// between the initial and the trained model, compilation).  Between launches
// the state lives in a training buffer of floats (train_buf_floats):
//   init[NP_PAD]                  the initial parameters
//   state[2][3][NP_PAD]           parameters, Adam's m1 and m2 after step k
//                                 in state[k & 1]
//   part[2][TRAIN_GMAX][NP_PAD]   per-workgroup gradients of the minibatch
//                                 of step s in part[s & 1]
//   lpart[2][LOSS_GMAX]           per-workgroup squared-error sums of the
//                                 strided loss, initial model in lpart[0],
//                                 final one in lpart[1]
constexpr int TRAIN_GMAX = 128;  // at most 128 * STEP_PTS = 32768 points per minibatch
constexpr int LOSS_PTS = 1024;   // strided-loss points per step workgroup
constexpr int LOSS_GMAX = 256;   // at most 2^18 strided points (m <= 2^24)

__device__ inline float* tb_init(float* tb) { return tb; }
__device__ inline float* tb_state(float* tb, int k) { return tb + NP_PAD + (size_t)(k & 1) * 3 * NP_PAD; }
__device__ inline float* tb_part(float* tb, int s) { return tb + 7 * NP_PAD + (size_t)(s & 1) * TRAIN_GMAX * NP_PAD; }
__device__ inline float* tb_loss(float* tb, int which)
{
    return tb + 7 * NP_PAD + 2 * (size_t)TRAIN_GMAX * NP_PAD + (size_t)which * LOSS_GMAX;
}

// Adam (Kingma and Ba 2015) with bias correction, step k counted from 1.
__device__ inline void adam_update(float& p, float& m1, float& m2, float g, int k, float lr)
{
    m1 = 0.9f * m1 + 0.1f * g;
    m2 = 0.999f * m2 + 0.001f * g * g;
    const float c1 = 1.f - powf(0.9f, (float)k);
    const float c2 = 1.f - powf(0.999f, (float)k);
    p -= lr * (m1 / c1) / (sqrtf(m2 / c2) + 1e-8f);
}

// x[0] + x[stride] + ... + x[(cnt - 1) * stride], added in that order; the
// loads are issued 16 at a time so that they overlap.
__device__ inline float ordered_sum(const float* x, int stride, int cnt)
{
    float sum = 0.f;
    int k = 0;
    for (; k + 16 <= cnt; k += 16) {
        float v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = x[(size_t)(k + q) * stride];
#pragma unroll
        for (int q = 0; q < 16; ++q) sum += v[q];
    }
    for (; k < cnt; ++k) sum += x[(size_t)k * stride];
    return sum;
}

// Hinges at H evenly spaced sample quantiles, slopes so that the model
// interpolates (i + 1/2)/m there.
template <int H>
__global__ __launch_bounds__(256) void k_cdf_init(const float* __restrict__ u, uint64_t m, float* tb)
{
    __shared__ float q[VMPS_CDF_MAX_HIDDEN], y[VMPS_CDF_MAX_HIDDEN], p[3 * VMPS_CDF_MAX_HIDDEN + 1];
    const int t = threadIdx.x;
    constexpr int NP = 3 * H + 1;
    if (t < H) {
        const uint64_t qi = (H > 1) ? ((uint64_t)t * (m - 1)) / (H - 1) : 0;
        q[t] = u[qi];
        y[t] = ((float)qi + 0.5f) / (float)m;
    }
    __syncthreads();
    if (t == 0)
        for (int h = 1; h < H; ++h)
            if (q[h] <= q[h - 1]) q[h] = q[h - 1] + KNOT_GAP;
    __syncthreads();
    if (t < H) {
        const float right = (t + 1 < H) ? (y[t + 1] - y[t]) / (q[t + 1] - q[t]) : 0.f;
        const float left = (t > 0) ? (y[t] - y[t - 1]) / (q[t] - q[t - 1]) : 0.f;
        p[t] = 1.f;
        p[H + t] = -q[t];
        p[2 * H + t] = right - left;
    }
    if (t == 0) p[3 * H] = y[0];
    __syncthreads();
    if (t < NP) {
        float* st = tb_state(tb, 0);
        tb_init(tb)[t] = p[t];
        st[t] = p[t];
        st[NP_PAD + t] = 0.f;
        st[2 * NP_PAD + t] = 0.f;
    }
}

// Launch s of the chain (s = 0 .. steps): the parameters after Adam step s
// (for s > 0 every workgroup applies the same update with the gradient of
// minibatch s - 1, its workgroup parts summed in workgroup order, and
// workgroup 0 stores the new state); then, for s < steps, this workgroup's
// part of the gradient of minibatch s (points [blockIdx.x * STEP_PTS, ...)
// of the nb points ((s nb + j) * stride) mod m); and for s = 0 (initial
// model) and s = steps (final model), this workgroup's part of the squared
// error over every LOSS_STRIDE-th sample point.
template <int H>
__global__ __launch_bounds__(STEP_NT) void k_cdf_step(const float* __restrict__ u, uint64_t m, int s, int steps,
                                                      int nb, float lr, float* tb)
{
    __shared__ TrainLds<STEP_NT> S;
    static_assert(STEP_NT >= 3 * VMPS_CDF_MAX_HIDDEN + 1, "one thread per parameter");
    const int t = threadIdx.x;
    constexpr int NP = 3 * H + 1;
    const int G = (nb + STEP_PTS - 1) / STEP_PTS;
    float gsum = 0.f;
    if (s > 0 && t < NP) gsum = ordered_sum(tb_part(tb, s - 1) + t, NP_PAD, G);
    if (t < NP) {
        const float* prev = tb_state(tb, s > 0 ? s - 1 : 0);
        float p = prev[t];
        if (s > 0) {
            float m1 = prev[NP_PAD + t], m2 = prev[2 * NP_PAD + t];
            adam_update(p, m1, m2, gsum, s, lr);
            if (blockIdx.x == 0) {
                float* st = tb_state(tb, s);
                st[t] = p;
                st[NP_PAD + t] = m1;
                st[2 * NP_PAD + t] = m2;
            }
        }
        S.p[t] = p;
    }
    __syncthreads();
    const int j0 = (int)blockIdx.x * STEP_PTS;
    if (s < steps && j0 < nb) {
        const int cnt = nb - j0 < STEP_PTS ? nb - j0 : STEP_PTS;
        const float fm = (float)m;
        batch_grad<H, STEP_NT>(S, cnt, 2.f / (float)nb, [&](int j, float& uu, float& yy) {
            const uint64_t idx = (((uint64_t)s * (uint64_t)nb + (uint64_t)(j0 + j)) * BATCH_STRIDE) % m;
            uu = u[idx];
            yy = ((float)idx + 0.5f) / fm;
        });
        if (t < NP) tb_part(tb, s)[(size_t)blockIdx.x * NP_PAD + t] = S.g[t];
    }
    if (s == 0 || s == steps) {
        const uint64_t cnt = (m + LOSS_STRIDE - 1) / LOSS_STRIDE;
        const uint64_t k0 = (uint64_t)blockIdx.x * LOSS_PTS;
        float acc = 0.f;
        for (uint64_t k = k0 + t; k < k0 + LOSS_PTS && k < cnt; k += STEP_NT) {
            const uint64_t i = k * LOSS_STRIDE;
            const float e = model_eval<H>(S.p, u[i]) - ((float)i + 0.5f) / (float)m;
            acc += e * e;
        }
        // fixed order: a butterfly inside each wave, then the waves in order
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
        if ((t & 63) == 0) S.pl[t >> 6] = acc;
        __syncthreads();
        if (t == 0 && k0 < cnt) {
            float sum = 0.f;
            for (int w = 0; w < STEP_NT / 64; ++w) sum += S.pl[w];
            if (s == 0) tb_loss(tb, 0)[blockIdx.x] = sum;
            if (s == steps) tb_loss(tb, 1)[blockIdx.x] = sum;
        }
    }
}

// The choice between the initial and the trained model by their strided
// losses (or the trained one when keep_trained is set), and the
// compilation of the chosen parameters into the knot table.
template <int H>
__global__ __launch_bounds__(TRAIN_NT) void k_cdf_finish(uint64_t m, int steps, int K, int keep_trained, float* tb,
                                                         vmps_cdf_model* model)
{
    __shared__ float p[3 * VMPS_CDF_MAX_HIDDEN + 1];
    __shared__ float losses[2];
    __shared__ uint32_t scan_lds[TRAIN_NT];
    const int t = threadIdx.x;
    constexpr int NP = 3 * H + 1;
    const uint64_t cnt = (m + LOSS_STRIDE - 1) / LOSS_STRIDE;
    const int GL = (int)((cnt + LOSS_PTS - 1) / LOSS_PTS);
    if (t < 2) losses[t] = ordered_sum(tb_loss(tb, t), 1, GL) / (float)cnt;
    __syncthreads();
    const float loss0 = losses[0], loss1 = losses[1];
    const bool keep = !keep_trained && !(loss1 <= loss0);
    if (t < NP) p[t] = keep ? tb_init(tb)[t] : tb_state(tb, steps)[t];
    if (t == 0) {
        model->trained = keep ? 0 : 1;
        model->loss_init = loss0;
        model->loss_final = keep ? loss0 : loss1;
    }
    __syncthreads();
    compile_table<H>(p, model, model->z_lo, model->z_hi, K, scan_lds);
}

// ------------------------------------------------------------ buckets --
template <typename K>
__global__ void k_bucket_ids(const K* __restrict__ keys, uint64_t n, const vmps_cdf_model* __restrict__ model,
                             uint32_t B, uint32_t* __restrict__ ids)
{
    const ModelArgs M = model_args(model, B);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        ids[i] = bucket_of((uint64_t)keys[i], M);
}

// One level of the stable scatter: parents [pstart[c], pstart[c+1]) are cut
// into tiles (tile prefix tbase); digit = (bucket >> shift) & mask.
struct PartLevel {
    const uint32_t* pstart;
    const uint32_t* tbase;
    uint32_t P, F, shift, mask, dbits;
    uint32_t* counts;
    const uint32_t* offs;
};

// Workgroups are dealt to the 8 XCDs in turn; this numbering gives every
// XCD a contiguous range of tiles, so the partly written cache lines where
// one tile's digit run meets the next tile's are completed in one L2.
__device__ inline uint32_t xcd_tile(uint32_t b, uint32_t G)
{
    const uint32_t x = b & 7, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

__device__ inline void part_tile(const PartLevel& L, uint32_t tile, uint32_t& c, uint32_t& tl, uint32_t& nt,
                                 uint32_t& s0, uint32_t& s1)
{
    uint32_t lo = 0, hi = L.P;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (L.tbase[mid] <= tile) lo = mid; else hi = mid;
    }
    c = lo;
    tl = tile - L.tbase[c];
    nt = L.tbase[c + 1] - L.tbase[c];
    s0 = L.pstart[c] + tl * PART_TILE;
    s1 = min(L.pstart[c + 1], s0 + PART_TILE);
}

// The model's knot table in LDS as 32-bit values when it is monotone and
// fits 32 bits (a compiled table always does): then buckets come from
// bucket_of32; otherwise (fast = false) from the 64-bit evaluation that
// reads the table in global memory.  Block-wide.
struct PartModel {
    ModelArgs M;
    ModelArgs32 M32;
    bool fast;
    __device__ uint32_t bucket(uint64_t key) const { return fast ? bucket_of32(key, M32) : bucket_of(key, M); }
};

__device__ inline PartModel part_model(const vmps_cdf_model* model, uint32_t B, uint32_t* tab)
{
    PartModel P;
    P.M = model_args(model, B);
    bool bad = false;
    for (int i = threadIdx.x; i <= P.M.knots; i += blockDim.x) {
        const uint64_t t = P.M.table[i];
        tab[i] = (uint32_t)t;
        bad |= (t >> 32) != 0 || (i > 0 && P.M.table[i - 1] > t);
    }
    P.fast = !__syncthreads_or(bad);
    P.M32 = model_args32(P.M, tab);
    return P;
}

// The per-tile counts of a histogram level go to a digit-major table (digit
// d of tile t at d * tiles + t, the order the offsets scan needs), one word
// per digit and tile.  Written tile by tile, every word is a partial write
// of its own 32-byte sector, from whichever XCD ran the tile (0.54 GB of
// sector traffic per level for 68 MB of counts at n = 2^28).  So a
// workgroup takes HIST_CHUNK consecutive tiles, keeps their counts in LDS
// (16 bits each: a tile holds at most 8192 keys) and then writes each
// digit's counts of those tiles together: consecutive words, from one XCD.
constexpr int HIST_CHUNK = 8;

// Level-2 histogram of HIST_CHUNK consecutive tiles from the 16-bit ids (the
// bucket's level-2 digit) the level-1 scatter moved with the keys.  Counting
// only, so the order is free: 16-byte chunks of 8 ids from the aligned
// position below s0 (the id arrays are padded to a multiple of 128), ids
// outside [s0, s1) skipped.  Per-wave counters keep LDS atomics on popular
// digits apart.
__global__ __launch_bounds__(PART_NT) void k_part_hist2(const uint16_t* __restrict__ ids_in, PartLevel L)
{
    __shared__ uint32_t hist[PART_NW][PART_DMAX];
    __shared__ uint16_t cbuf[HIST_CHUNK][PART_DMAX];
    __shared__ uint32_t cbase[HIST_CHUNK], cnt_t[HIST_CHUNK];
    const uint32_t ntiles = L.tbase[L.P];
    const uint32_t t0 = blockIdx.x * HIST_CHUNK;
    if (t0 >= ntiles) return;
    const uint32_t nc = ntiles - t0 < (uint32_t)HIST_CHUNK ? ntiles - t0 : (uint32_t)HIST_CHUNK;
    const int tid = threadIdx.x, wave = tid >> 6;
    for (uint32_t j = 0; j < nc; ++j) {
        uint32_t c, tl, nt, s0, s1;
        part_tile(L, t0 + j, c, tl, nt, s0, s1);
        for (int i = tid; i < PART_NW * PART_DMAX; i += PART_NT) (&hist[0][0])[i] = 0;
        __syncthreads();
        const uint32_t a0 = s0 & ~7u;
        const uint32_t chunks = (s1 - a0 + 7) / 8;
        for (uint32_t q = tid; q < chunks; q += PART_NT) {
            const uint4 w = *(const uint4*)(ids_in + a0 + 8 * q);
            const uint32_t word[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t idx = a0 + 8 * q + e;
                const uint32_t id = (word[e >> 1] >> (16 * (e & 1))) & 0xffffu;
                if (idx >= s0 && idx < s1) atomicAdd(&hist[wave][(id >> L.shift) & L.mask], 1u);
            }
        }
        __syncthreads();
        for (uint32_t d = tid; d < L.F; d += PART_NT) {
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < PART_NW; ++w) t += hist[w][d];
            cbuf[j][d] = (uint16_t)t;
        }
        if (tid == 0) {
            cbase[j] = L.tbase[c] * L.F + tl;
            cnt_t[j] = nt;
        }
        __syncthreads();
    }
    for (uint32_t d = tid; d < L.F; d += PART_NT)
        for (uint32_t j = 0; j < nc; ++j) L.counts[(uint64_t)cbase[j] + (uint64_t)d * cnt_t[j]] = cbuf[j][d];
}

// Level-1 histogram with the model: the level's tiles are the aligned
// PART_TILE blocks of the whole array.  Each workgroup copies the knot
// table into LDS once and then takes tiles tile, tile + grid, ...; keys
// are read two at a time.  Every key's bucket id goes out for the level-1
// scatter: its low 16 bits in ids_out (staged in LDS in tile order, then
// 16 bytes per lane), and for B > 2^16 its bits 16 and 17 in hibits (bits
// 2(i mod 16), 2(i mod 16) + 1 of word i / 16 for key i).
template <typename K>
__global__ __launch_bounds__(PART_NT) void k_part_hist1(const K* __restrict__ keys, uint16_t* __restrict__ ids_out,
                                                        uint32_t* __restrict__ hibits, uint32_t n, uint32_t nt1,
                                                        uint32_t F, uint32_t shift, uint32_t mask,
                                                        uint32_t* __restrict__ counts,
                                                        const vmps_cdf_model* __restrict__ model, uint32_t B)
{
    struct alignas(2 * sizeof(K)) KPair { K a, b; };
    constexpr int RP = PART_RND / 2;  // key pairs per thread
    __shared__ uint32_t tab[VMPS_CDF_MAX_KNOTS + 1];
    __shared__ uint32_t hist[PART_NW][PART_DMAX];
    __shared__ __align__(16) uint32_t stage[PART_TILE];  // bucket ids in tile order
    __shared__ uint16_t cbuf[HIST_CHUNK][PART_DMAX];      // counts of the chunk's tiles
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const PartModel PM = part_model(model, B, tab);
    const bool hi = B > 65536;
    const uint32_t nch = (nt1 + HIST_CHUNK - 1) / HIST_CHUNK;
    for (uint32_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const uint32_t tc0 = ch * HIST_CHUNK;
        const uint32_t nc = nt1 - tc0 < (uint32_t)HIST_CHUNK ? nt1 - tc0 : (uint32_t)HIST_CHUNK;
        for (uint32_t jt = 0; jt < nc; ++jt) {
            const uint32_t tile = tc0 + jt;
            for (int i = tid; i < PART_NW * PART_DMAX; i += PART_NT) (&hist[0][0])[i] = 0;
            __syncthreads();
            const uint32_t s0 = tile * PART_TILE;
            const uint32_t len = n - s0 < PART_TILE ? n - s0 : PART_TILE;
            KPair kp[RP];
#pragma unroll
            for (int r = 0; r < RP; ++r) {
                const uint32_t q = 2 * (r * PART_NT + tid);
                if (q + 1 < len) {
                    kp[r] = *(const KPair*)(keys + s0 + q);
                } else {
                    kp[r].a = q < len ? keys[s0 + q] : K(0);
                    kp[r].b = K(0);
                }
            }
#pragma unroll
            for (int r = 0; r < RP; ++r) {
                const uint32_t q = 2 * (r * PART_NT + tid);
                if (q < len) {
                    const uint32_t b0 = PM.bucket((uint64_t)kp[r].a);
                    atomicAdd(&hist[wave][(b0 >> shift) & mask], 1u);
                    stage[q] = b0;
                }
                if (q + 1 < len) {
                    const uint32_t b1 = PM.bucket((uint64_t)kp[r].b);
                    atomicAdd(&hist[wave][(b1 >> shift) & mask], 1u);
                    stage[q + 1] = b1;
                }
            }
            __syncthreads();
            if ((uint32_t)tid < F) {
                uint32_t t = 0;
#pragma unroll
                for (int w = 0; w < PART_NW; ++w) t += hist[w][tid];
                cbuf[jt][tid] = (uint16_t)t;  // each thread keeps its own digit's column
            }
            // ids out: lane t of the workgroup holds keys [8t, 8t + 8) of the
            // tile per round (PART_TILE / 8 / PART_NT rounds)
#pragma unroll
            for (int r = 0; r < (int)(PART_TILE / 8 / PART_NT); ++r) {
                const uint32_t e = 8 * (r * PART_NT + tid);
                const uint4 lo4 = *(const uint4*)&stage[e], hi4 = *(const uint4*)&stage[e + 4];
                const uint32_t bs[8] = {lo4.x, lo4.y, lo4.z, lo4.w, hi4.x, hi4.y, hi4.z, hi4.w};
                uint32_t w[4] = {0u, 0u, 0u, 0u}, hb = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint32_t b = e + j < len ? bs[j] : 0u;
                    w[j >> 1] |= (b & 0xffffu) << (16 * (j & 1));
                    hb |= ((b >> 16) & 3u) << (2 * j);
                }
                if (e + 8 <= len) {
                    *(uint4*)(ids_out + s0 + e) = make_uint4(w[0], w[1], w[2], w[3]);
                } else {
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (e + j < len) ids_out[s0 + e + j] = (uint16_t)(w[j >> 1] >> (16 * (j & 1)));
                }
                if (hi) {
                    // two lanes make one 16-key word (the tile start is a
                    // multiple of 16); lanes past the end contribute zeros
                    uint32_t word = hb << (16 * (lane & 1));
                    word |= __shfl_xor(word, 1, 64);
                    if ((lane & 1) == 0 && e < len) hibits[(s0 + e) >> 4] = word;
                }
            }
            __syncthreads();
        }
        // the chunk's counts, digit by digit: nc consecutive words per digit
        if ((uint32_t)tid < F)
            for (uint32_t jt = 0; jt < nc; ++jt) counts[(uint64_t)tid * nt1 + tc0 + jt] = cbuf[jt][tid];
    }
}

// LDS of one scatter workgroup: the tile goes back out in NPART parts.
template <typename K, int VMODE, int LEVEL>
struct ScatterLds {
    static constexpr int NPART = (LEVEL == 1 && VMODE) ? 4 : 2;
    static constexpr uint32_t PARTN = PART_TILE / NPART;
    static constexpr int D = PART_DMAX;  // digits of the level: at most 9 bits
    using Sid = typename std::conditional<LEVEL == 1, uint32_t, uint16_t>::type;
    K skey[PARTN];
    uint32_t sval[VMODE ? PARTN : 1];
    Sid sid[PARTN];
    uint32_t hc[PART_NW][D];
    uint32_t loff[D], goff[D];
    uint32_t scan[PART_NW + 1];
    uint32_t hib[LEVEL == 1 ? PART_TILE / 16 : 1];  // bits 16-17 of the tile's bucket ids
};

// Stable scatter of one tile by the digit of its bucket id.  Wave w ranks
// the keys [w*TILE/NW, (w+1)*TILE/NW) of the tile in input order: a match
// of the digit bits by ballots gives the rank among the wave's 64 keys, a
// wave-private counter per digit the rank among its earlier keys.  One
// block scan over (digit, wave) gives every key its place in an LDS reorder
// by digit, and the runs of equal digit go out contiguously.  The reorder
// goes through LDS in parts of the tile, so that two workgroups share a
// CU.  VMODE 2 generates the values (input index).
//   LEVEL 1: the whole array in aligned tiles; every key's bucket id comes
//     from the level-1 histogram (16-bit ids, and bits 16-17 from hibits
//     when it is not null); the bucket's level-2 digit goes out with the
//     key as a 16-bit id.
//   LEVEL 2: the tiles of every level-1 range; the digit is the 16-bit id.
// A key's bucket (18 bits at most) and its place in the tile (13 bits) share
// one 32-bit register: bucket below, place from bit 18.
template <typename K, int VMODE, int LEVEL>
__device__ inline void scatter_tile(ScatterLds<K, VMODE, LEVEL>& S, const uint32_t* __restrict__ hibits,
                                    const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                    const uint16_t* __restrict__ idin, K* __restrict__ kout,
                                    uint32_t* __restrict__ vout, uint16_t* __restrict__ idout, const PartLevel& L,
                                    uint32_t tile, uint32_t id_mask)
{
    using SL = ScatterLds<K, VMODE, LEVEL>;
    constexpr uint32_t WCH = PART_TILE / PART_NW;  // keys per wave
    constexpr int RND = (int)(WCH / 64);
    constexpr uint32_t BMASK = (1u << 18) - 1;
    uint32_t c, tl, nt, s0, s1;
    part_tile(L, tile, c, tl, nt, s0, s1);
    const uint32_t len = s1 - s0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < PART_NW * SL::D; i += PART_NT) (&S.hc[0][0])[i] = 0;
    for (uint32_t d = tid; d < L.F; d += PART_NT) S.goff[d] = L.offs[(uint64_t)L.tbase[c] * L.F + (uint64_t)d * nt + tl];
    // level 1 beyond 2^16 buckets: the words holding bits 16-17 of the
    // tile's ids into LDS (the tile start is a multiple of 16)
    static_assert(PART_TILE / 16 <= PART_NT, "one word per thread");
    if (LEVEL == 1 && hibits && (uint32_t)tid < (len + 15) / 16) S.hib[tid] = hibits[(s0 >> 4) + tid];
    __syncthreads();

    const uint32_t wb = wave * WCH;
    K kr[RND];
    uint32_t vr[RND], ir[RND];
#pragma unroll
    for (int r = 0; r < RND; ++r) {
        const uint32_t i = wb + r * 64 + lane;
        const bool valid = i < len;
        kr[r] = valid ? kin[s0 + i] : K(0);
        ir[r] = valid ? idin[s0 + i] : 0u;
        vr[r] = (VMODE == 1 && valid) ? vin[s0 + i] : s0 + i;
    }
    if (LEVEL == 1 && hibits) {
#pragma unroll
        for (int r = 0; r < RND; ++r) {
            const uint32_t i = wb + r * 64 + lane;
            if (i < len) ir[r] |= ((S.hib[i >> 4] >> (2 * (i & 15))) & 3u) << 16;
        }
    }
    const uint64_t lt = (1ull << lane) - 1;
#pragma unroll
    for (int r = 0; r < RND; ++r) {
        const uint32_t i = wb + r * 64 + lane;
        const bool valid = i < len;
        const uint32_t d = valid ? (ir[r] >> L.shift) & L.mask : 0u;
        const uint64_t vb = __ballot(valid);
        uint32_t plo = (uint32_t)vb, phi = (uint32_t)(vb >> 32);
        for (uint32_t k = 0; k < L.dbits; ++k) {
            // nb = -bit (all ones or zero); the lanes agreeing with this lane
            // on bit k are ~(ballot ^ nb).  One bit-field extract and one
            // three-input bitwise operation per half: p & ~(b ^ c) has the
            // truth table 0x90 (operands 0xF0, 0xCC, 0xAA).
            const int nb = __builtin_amdgcn_sbfe((int)d, k, 1u);
            const uint64_t bk = __ballot(nb != 0);
            plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)bk, (uint32_t)nb, 0x90);
            phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(bk >> 32), (uint32_t)nb, 0x90);
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t before = valid ? S.hc[wave][d] : 0u;
        const uint32_t rw = __popcll(peers & lt);
        ir[r] |= (before + rw) << 18;
        // the wave's lowest lane of each digit advances the counter; LDS
        // operations of one wave complete in order, after every lane's read
        if (valid && rw == 0) S.hc[wave][d] = before + __popcll(peers);
    }
    __syncthreads();
    static_assert(SL::D <= PART_NT, "one digit per thread");
    uint32_t tot = 0;
    if (tid < SL::D) {
#pragma unroll
        for (int w = 0; w < PART_NW; ++w) {
            const uint32_t v = S.hc[w][tid];
            S.hc[w][tid] = tot;
            tot += v;
        }
    }
    uint32_t all;
    const uint32_t ex = block_excl_scan(tot, S.scan, &all);
    if (tid < SL::D) {
        S.loff[tid] = ex;
#pragma unroll
        for (int w = 0; w < PART_NW; ++w) S.hc[w][tid] += ex;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RND; ++r) {
        const uint32_t d = ((ir[r] & BMASK) >> L.shift) & L.mask;
        ir[r] += S.hc[wave][d] << 18;  // place in the tile's order by digit
    }
#pragma unroll
    for (uint32_t h = 0; h < (uint32_t)SL::NPART; ++h) {
        const uint32_t lo = h * SL::PARTN;
        if (lo >= len) break;
#pragma unroll
        for (int r = 0; r < RND; ++r) {
            const uint32_t i = wb + r * 64 + lane;
            const uint32_t lp = (ir[r] >> 18) - lo;
            if (i < len && lp < SL::PARTN) {
                S.skey[lp] = kr[r];
                S.sid[lp] = (typename SL::Sid)(ir[r] & BMASK);
                if (VMODE) S.sval[lp] = vr[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < (int)(SL::PARTN / PART_NT); ++r) {
            const uint32_t j = r * PART_NT + tid, i = lo + j;
            if (i < len) {
                const uint32_t id = S.sid[j];
                const uint32_t d = (id >> L.shift) & L.mask;
                const uint32_t o = S.goff[d] + (i - S.loff[d]);
                kout[o] = S.skey[j];
                if (VMODE) vout[o] = S.sval[j];
                if (LEVEL == 1) idout[o] = (uint16_t)(id & id_mask);
            }
        }
        __syncthreads();
    }
}

template <typename K, int VMODE>
__global__ __launch_bounds__(PART_NT, 4) void k_part_scatter1(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                           const uint16_t* __restrict__ idin,
                                                           const uint32_t* __restrict__ hibits, K* __restrict__ kout,
                                                           uint32_t* __restrict__ vout, uint16_t* __restrict__ idout,
                                                           PartLevel L, uint32_t id_mask)
{
    __shared__ ScatterLds<K, VMODE, 1> S;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    scatter_tile<K, VMODE, 1>(S, hibits, kin, vin, idin, kout, vout, idout, L, tile, id_mask);
}

template <typename K, int VMODE>
__global__ __launch_bounds__(PART_NT, 4) void k_part_scatter2(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                           const uint16_t* __restrict__ idin, K* __restrict__ kout,
                                                           uint32_t* __restrict__ vout, PartLevel L)
{
    __shared__ ScatterLds<K, VMODE, 2> S;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= L.tbase[L.P]) return;
    scatter_tile<K, VMODE, 2>(S, nullptr, kin, vin, idin, kout, vout, nullptr, L, tile, 0u);
}

// Level-1 parents: the whole array.
__global__ void k_part_init(uint32_t n, uint32_t* pstart, uint32_t* tbase, uint32_t* count_out, uint32_t F)
{
    pstart[0] = 0;
    pstart[1] = n;
    tbase[0] = 0;
    tbase[1] = (uint32_t)ceil_div(n, PART_TILE);
    *count_out = tbase[1] * F;
}

// Level-2 parents: the level-1 digit ranges.
__global__ __launch_bounds__(PART_DMAX) void k_part_level2(const uint32_t* __restrict__ offs1, uint32_t nt1,
                                                           uint32_t F1, uint32_t n, uint32_t F2,
                                                           uint32_t* __restrict__ pstart, uint32_t* __restrict__ tbase,
                                                           uint32_t* count_out)
{
    __shared__ uint32_t lds[PART_DMAX / WAVE + 1];
    const uint32_t c = threadIdx.x;
    uint32_t s = 0, e = 0;
    if (c < F1) {
        s = offs1[(uint64_t)c * nt1];
        e = (c + 1 < F1) ? offs1[(uint64_t)(c + 1) * nt1] : n;
        pstart[c] = s;
    }
    if (c == 0) pstart[F1] = n;
    const uint32_t tiles = c < F1 ? (uint32_t)ceil_div(e - s, PART_TILE) : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(tiles, lds, &tot);
    if (c < F1) tbase[c] = ex;
    if (c == 0) { tbase[F1] = tot; *count_out = tot * F2; }
}

__global__ void k_zero_offsets(int64_t* off, uint32_t B)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b <= B) off[b] = 0;
}

// Start of every bucket after both levels.
__global__ void k_bucket_offsets(const uint32_t* __restrict__ pstart2, const uint32_t* __restrict__ tbase2,
                                 const uint32_t* __restrict__ offs2, uint32_t F2, uint32_t lo_bits, uint32_t B,
                                 uint32_t n, int64_t* __restrict__ off)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > B) return;
    if (b == B) { off[B] = n; return; }
    const uint32_t c = b >> lo_bits, f = b & ((1u << lo_bits) - 1);
    const uint32_t nt = tbase2[c + 1] - tbase2[c];
    off[b] = nt ? offs2[(uint64_t)tbase2[c] * F2 + (uint64_t)f * nt] : pstart2[c];
}

// Error judge of the compiled model on the sorted sample x_0..x_{m-1},
// targets y_i = (i + 1/2)/m.  Per point: the bucket error
// |bucket(x_i) - floor(B y_i)| and the exact numerator
// d_i = |2m F(x_i) 2^32 - 2^32 (2i+1)| of the CDF error B d_i / (2^33 m).
// Each workgroup writes its maxima and sums (128-bit as two words) to
// part[6 * blockIdx.x ...]; k_learned_stats combines them.
typedef unsigned __int128 u128;

template <typename K>
__global__ __launch_bounds__(256) void k_learned_judge(const K* __restrict__ sample, uint64_t m,
                                                       const vmps_cdf_model* model, uint32_t B,
                                                       uint64_t* __restrict__ part)
{
    __shared__ uint64_t s_mb[256], s_sb[256];
    __shared__ u128 s_dm[256], s_ds[256];
    const ModelArgs M = model_args(model, B);
    uint64_t mb = 0, sb = 0;
    u128 dm = 0, ds = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (uint64_t)gridDim.x * 256) {
        const uint64_t pos = cdf_pos((uint64_t)sample[i], M);
        uint64_t b = (pos * B) >> 32;
        b = b >= B ? B - 1 : b;
        const uint64_t want = ((uint64_t)B * (2 * i + 1)) / (2 * m);
        const uint64_t eb = b > want ? b - want : want - b;
        mb = eb > mb ? eb : mb;
        sb += eb;
        const u128 a = (u128)pos * (u128)(2 * m);
        const u128 t = (u128)(2 * i + 1) << 32;
        const u128 d = a > t ? a - t : t - a;
        dm = d > dm ? d : dm;
        ds += d;
    }
    s_mb[threadIdx.x] = mb; s_sb[threadIdx.x] = sb; s_dm[threadIdx.x] = dm; s_ds[threadIdx.x] = ds;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            s_mb[threadIdx.x] = s_mb[o] > s_mb[threadIdx.x] ? s_mb[o] : s_mb[threadIdx.x];
            s_sb[threadIdx.x] += s_sb[o];
            s_dm[threadIdx.x] = s_dm[o] > s_dm[threadIdx.x] ? s_dm[o] : s_dm[threadIdx.x];
            s_ds[threadIdx.x] += s_ds[o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint64_t* p = part + 6 * (uint64_t)blockIdx.x;
        p[0] = s_mb[0]; p[1] = s_sb[0];
        p[2] = (uint64_t)s_dm[0]; p[3] = (uint64_t)(s_dm[0] >> 64);
        p[4] = (uint64_t)s_ds[0]; p[5] = (uint64_t)(s_ds[0] >> 64);
    }
}

__device__ inline double u128_to_double(u128 x)
{
    return (double)(uint64_t)(x >> 64) * 18446744073709551616.0 + (double)(uint64_t)x;
}

__global__ __launch_bounds__(256) void k_learned_stats(const int64_t* __restrict__ off, uint32_t B, uint32_t T,
                                                       const vmps_cdf_model* model, uint64_t m,
                                                       const uint64_t* __restrict__ part, vmps_learned_stats* st)
{
    __shared__ unsigned long long s_ne, s_fb, s_fk, s_mx;
    __shared__ uint64_t s_mb[JUDGE_GRID], s_sb[JUDGE_GRID];
    __shared__ u128 s_dm[JUDGE_GRID], s_ds[JUDGE_GRID];
    static_assert(JUDGE_GRID == 256, "one judge partial per thread");
    if (threadIdx.x == 0) { s_ne = 0; s_fb = 0; s_fk = 0; s_mx = 0; }
    {
        const uint64_t* p = part + 6 * threadIdx.x;
        s_mb[threadIdx.x] = p[0]; s_sb[threadIdx.x] = p[1];
        s_dm[threadIdx.x] = ((u128)p[3] << 64) | p[2];
        s_ds[threadIdx.x] = ((u128)p[5] << 64) | p[4];
    }
    __syncthreads();
    unsigned long long ne = 0, fb = 0, fk = 0, mx = 0;
    for (uint32_t b = threadIdx.x; b < B; b += 256) {
        const unsigned long long len = (unsigned long long)(off[b + 1] - off[b]);
        ne += len > 0;
        if (len > T) { fb += 1; fk += len; }
        mx = len > mx ? len : mx;
    }
    atomicAdd(&s_ne, ne); atomicAdd(&s_fb, fb); atomicAdd(&s_fk, fk); atomicMax(&s_mx, mx);
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            s_mb[threadIdx.x] = s_mb[o] > s_mb[threadIdx.x] ? s_mb[o] : s_mb[threadIdx.x];
            s_sb[threadIdx.x] += s_sb[o];
            s_dm[threadIdx.x] = s_dm[o] > s_dm[threadIdx.x] ? s_dm[o] : s_dm[threadIdx.x];
            s_ds[threadIdx.x] += s_ds[o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->buckets = B; st->nonempty_buckets = (int64_t)s_ne; st->fallback_buckets = (int64_t)s_fb;
        st->fallback_keys = (int64_t)s_fk; st->max_bucket = (int64_t)s_mx;
        st->loss_init = model->loss_init; st->loss_final = model->loss_final;
        const double dm = (double)m, denom = dm * 8589934592.0;  // 2^33 m
        st->judge_samples = (int64_t)m;
        st->judge_max_bucket_err = (int64_t)s_mb[0];
        st->judge_mean_bucket_err = (double)s_sb[0] / dm;
        st->judge_max_err = u128_to_double(s_dm[0]) * (double)B / denom;
        st->judge_mean_err = u128_to_double(s_ds[0]) * (double)B / denom / dm;
        st->overflow_fraction = (double)s_fb / (double)B;
    }
}

// Grouping of consecutive buckets for the bucket sort.  Buckets are
// increasing key ranges, so the stable sort of several consecutive buckets
// as one Powersort instance is the concatenation of their stable sorts:
// groups change only how the tile pass's workgroups are filled.  Greedy
// packing inside chunks of GROUP_CHUNK buckets (a chunk boundary is always a
// group boundary): a group takes the next bucket while its length stays
// within C; a bucket longer than C is a group of its own.
constexpr uint32_t GROUP_CHUNK = 64;

__device__ inline uint32_t group_chunk(const int64_t* __restrict__ boff, uint32_t B, uint32_t chunk, uint64_t C,
                                       int64_t* __restrict__ out)
{
    const uint32_t b0 = chunk * GROUP_CHUNK, b1 = min(B, b0 + GROUP_CHUNK);
    uint32_t cnt = 0;
    int64_t gs = boff[b0];
    for (uint32_t b = b0 + 1; b < b1; ++b) {
        const int64_t bs = boff[b], be = boff[b + 1];
        if ((uint64_t)(be - gs) > C && bs > gs) {  // bucket b does not fit a non-empty group
            if (out) out[cnt] = gs;
            ++cnt;
            gs = bs;
        }
    }
    if (out) out[cnt] = gs;
    return cnt + 1;
}

__global__ void k_group_count(const int64_t* __restrict__ boff, uint32_t B, uint64_t C, uint32_t* __restrict__ cnt)
{
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c * GROUP_CHUNK < B) cnt[c] = group_chunk(boff, B, c, C, nullptr);
}

__global__ void k_group_emit(const int64_t* __restrict__ boff, uint32_t B, uint64_t C,
                             const uint32_t* __restrict__ base, int64_t* __restrict__ goff)
{
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c * GROUP_CHUNK < B) group_chunk(boff, B, c, C, goff + base[c]);
}

// goff[G, B] = n, G = the number of groups
__global__ void k_group_pad(const uint32_t* __restrict__ total, uint32_t B, uint32_t n, int64_t* __restrict__ goff)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= B && i >= *total) goff[i] = n;
}

// ------------------------------------------------------------- host --
namespace {
inline unsigned grid1(uint64_t n, unsigned b = 256) { return (unsigned)ceil_div(n ? n : 1, b); }

// Bucket id bits: level 2 takes the low 9 bits from 2^17 buckets on, else
// the bits beyond the top 8; level 1 the rest (at most 9).
struct PartBits {
    uint32_t lo_bits, F1, F2;
};

inline PartBits part_bits(uint32_t B)
{
    uint32_t bits = 0;
    while ((1u << bits) < B) ++bits;
    PartBits p;
    p.lo_bits = bits >= 17 ? 9 : (bits > 8 ? bits - 8 : 0);
    p.F1 = B >> p.lo_bits;
    p.F2 = 1u << p.lo_bits;
    return p;
}

template <typename K>
hipError_t partition_t(const K* kin, const uint32_t* vin, K* ktmp, uint32_t* vtmp, K* kout, uint32_t* vout,
                       uint32_t n, int vmode, const vmps_cdf_model* Mdev, uint32_t B, int64_t* bucket_off,
                       uint32_t* arena, hipStream_t s)
{
    const PartBits pb = part_bits(B);
    const uint32_t lo_bits = pb.lo_bits, F1 = pb.F1, F2 = pb.F2;
    const uint32_t nt1 = (uint32_t)ceil_div(n, PART_TILE);
    const uint32_t nt2cap = nt1 + F1;
    uint32_t* p1 = arena;            // pstart1[2], tbase1[2]
    uint32_t* t1 = arena + 2;
    uint32_t* p2 = arena + 4;        // F1 + 1 <= 513
    uint32_t* t2 = p2 + 520;         // F1 + 1
    uint32_t* cnt_total = t2 + 520;  // 2 scalars
    uint32_t* tot = cnt_total + 2;   // 2 scalars
    uint32_t* c1 = tot + 4;
    uint32_t* o1 = c1 + (uint64_t)nt1 * F1;
    uint32_t* c2 = o1 + (uint64_t)nt1 * F1;
    uint32_t* o2 = c2 + (uint64_t)nt2cap * F2;
    uint32_t* stmp = o2 + (uint64_t)nt2cap * F2;
    const uint64_t big = (uint64_t)nt1 * F1 > (uint64_t)nt2cap * F2 ? (uint64_t)nt1 * F1 : (uint64_t)nt2cap * F2;
    uint16_t* id1 = (uint16_t*)(((uintptr_t)(stmp + scan_tmp_words(big)) + 255) & ~(uintptr_t)255);
    uint16_t* id2 = id1 + ((n + 127) & ~127u);
    uint32_t* hib = B > 65536 ? (uint32_t*)(id2 + ((n + 127) & ~127u)) : nullptr;  // (n + 15) / 16 words
    uint32_t dbits1 = 0, dbits2 = 0;
    while ((1u << dbits1) < F1) ++dbits1;
    while ((1u << dbits2) < F2) ++dbits2;
    // the level-1 histogram's grid is persistent: as many workgroups as are
    // resident at once (a second round would run on a mostly idle GPU)
    static bool occ_set[16] = {};
    static unsigned occ_h1[16] = {};
    int dev = 0;
    VMPS_HIP(hipGetDevice(&dev));
    const int d = dev & 15;
    if (!occ_set[d]) {
        int per_cu = 0, cus = 0;
        VMPS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_part_hist1<K>, PART_NT, 0));
        VMPS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        occ_h1[d] = (unsigned)((per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1));
        occ_set[d] = true;
    }
    {
        TraceScope tr(VMPS_TRACE_HISTOGRAM, s);
        k_part_init<<<1, 1, 0, s>>>(n, p1, t1, cnt_total, F1);
        const uint32_t nch1 = (uint32_t)ceil_div(nt1, HIST_CHUNK);
        const unsigned g1 = nch1 < occ_h1[d] ? nch1 : occ_h1[d];
        k_part_hist1<K><<<g1, PART_NT, 0, s>>>(kin, id1, hib, n, nt1, F1, lo_bits, F1 - 1, c1, Mdev, B);
        VMPS_HIP(scan_exclusive_u32(c1, o1, (uint64_t)nt1 * F1, cnt_total, tot, stmp, s));
    }
    {
        TraceScope tr(VMPS_TRACE_SCATTER, s);
        PartLevel L1{p1, t1, 1, F1, lo_bits, F1 - 1, dbits1, c1, o1};
        const uint32_t idm = F2 - 1;
        if (vmode == 0) k_part_scatter1<K, 0><<<nt1, PART_NT, 0, s>>>(kin, vin, id1, hib, ktmp, vtmp, id2, L1, idm);
        else if (vmode == 1) k_part_scatter1<K, 1><<<nt1, PART_NT, 0, s>>>(kin, vin, id1, hib, ktmp, vtmp, id2, L1, idm);
        else k_part_scatter1<K, 2><<<nt1, PART_NT, 0, s>>>(kin, vin, id1, hib, ktmp, vtmp, id2, L1, idm);
    }
    {
        TraceScope tr(VMPS_TRACE_HISTOGRAM, s);
        k_part_level2<<<1, PART_DMAX, 0, s>>>(o1, nt1, F1, n, F2, p2, t2, cnt_total + 1);
        PartLevel L2{p2, t2, F1, F2, 0, F2 - 1, dbits2, c2, o2};
        k_part_hist2<<<(unsigned)ceil_div(nt2cap, HIST_CHUNK), PART_NT, 0, s>>>(id2, L2);
        VMPS_HIP(scan_exclusive_u32(c2, o2, (uint64_t)nt2cap * F2, cnt_total + 1, tot + 1, stmp, s));
    }
    {
        TraceScope tr(VMPS_TRACE_SCATTER, s);
        PartLevel L2{p2, t2, F1, F2, 0, F2 - 1, dbits2, c2, o2};
        if (vmode == 0) k_part_scatter2<K, 0><<<nt2cap, PART_NT, 0, s>>>(ktmp, vtmp, id2, kout, vout, L2);
        else k_part_scatter2<K, 1><<<nt2cap, PART_NT, 0, s>>>(ktmp, vtmp, id2, kout, vout, L2);
    }
    k_bucket_offsets<<<grid1(B + 1), 256, 0, s>>>(p2, t2, o2, F2, lo_bits, B, n, bucket_off);
    return hipGetLastError();
}
}  // namespace

uint64_t partition_arena_words(uint64_t n, uint32_t B)
{
    const PartBits pb = part_bits(B);
    const uint64_t F1 = pb.F1, F2 = pb.F2;
    const uint64_t nt1 = ceil_div(n ? n : 1, PART_TILE);
    const uint64_t nt2cap = nt1 + F1;
    const uint64_t big = nt1 * F1 > nt2cap * F2 ? nt1 * F1 : nt2cap * F2;
    // two arrays of 16-bit ids (level-1 bucket ids, level-2 digits), and
    // bits 16-17 of the bucket ids beyond 2^16 buckets
    const uint64_t ids = 2 * ((n + 127) & ~127ull) / 2 + (B > 65536 ? (n + 15) / 16 + 4 : 0);
    return 4 + 1040 + 8 + 2 * nt1 * F1 + 2 * nt2cap * F2 + scan_tmp_words(big) + 64 + ids + 64;
}

uint64_t group_scratch_words(uint32_t B)
{
    const uint64_t nc = ceil_div(B ? B : 1, GROUP_CHUNK);
    return 2 * nc + 8 + scan_tmp_words(nc);
}

const uint32_t* group_count(const uint32_t* scratch, uint32_t B)
{
    return scratch + 2 * ceil_div(B, GROUP_CHUNK);
}

hipError_t group_enqueue(const int64_t* boff, uint32_t B, uint32_t n, uint32_t C, int64_t* goff, uint32_t* scratch,
                         hipStream_t s)
{
    const uint32_t nc = (uint32_t)ceil_div(B, GROUP_CHUNK);
    uint32_t* cnt = scratch;
    uint32_t* base = cnt + nc;
    uint32_t* tot = base + nc;  // 8 words
    uint32_t* tmp = tot + 8;
    k_group_count<<<grid1(nc), 256, 0, s>>>(boff, B, C, cnt);
    VMPS_HIP(scan_exclusive_u32(cnt, base, nc, nullptr, tot, tmp, s));
    k_group_emit<<<grid1(nc), 256, 0, s>>>(boff, B, C, base, goff);
    k_group_pad<<<grid1((uint64_t)B + 1), 256, 0, s>>>(tot, B, n, goff);
    return hipGetLastError();
}

hipError_t partition_enqueue(const void* kin, const uint32_t* vin, void* ktmp, uint32_t* vtmp, void* kout,
                             uint32_t* vout, uint32_t n, int key_bits, int vmode, const vmps_cdf_model* model,
                             uint32_t B, int64_t* bucket_off, uint32_t* arena, hipStream_t s)
{
    if (n == 0) {
        k_zero_offsets<<<grid1(B + 1), 256, 0, s>>>(bucket_off, B);
        return hipGetLastError();
    }
    if (key_bits == 32)
        return partition_t<uint32_t>((const uint32_t*)kin, vin, (uint32_t*)ktmp, vtmp, (uint32_t*)kout, vout, n,
                                     vmode, model, B, bucket_off, arena, s);
    return partition_t<uint64_t>((const uint64_t*)kin, vin, (uint64_t*)ktmp, vtmp, (uint64_t*)kout, vout, n, vmode,
                                 model, B, bucket_off, arena, s);
}

hipError_t sample_enqueue(const void* keys, uint64_t n, int key_bits, uint64_t m, uint64_t seed, void* out,
                          hipStream_t s)
{
    if (key_bits == 32)
        k_sample_gather<uint32_t><<<grid1(m), 256, 0, s>>>((const uint32_t*)keys, n, m, seed, (uint32_t*)out);
    else
        k_sample_gather<uint64_t><<<grid1(m), 256, 0, s>>>((const uint64_t*)keys, n, m, seed, (uint64_t*)out);
    return hipGetLastError();
}

uint64_t train_buf_floats() { return 7ull * NP_PAD + 2ull * TRAIN_GMAX * NP_PAD + 2ull * LOSS_GMAX; }

template <int H>
static void train_launches(const float* u, uint64_t m, const vmps_learned_config& c, float* tb, vmps_cdf_model* model,
                           hipStream_t s)
{
    k_cdf_init<H><<<1, 256, 0, s>>>(u, m, tb);
    const unsigned Gg = (unsigned)((c.batch + STEP_PTS - 1) / STEP_PTS);
    const uint64_t lcnt = (m + LOSS_STRIDE - 1) / LOSS_STRIDE;
    const unsigned Gl = (unsigned)((lcnt + LOSS_PTS - 1) / LOSS_PTS);
    for (int st = 0; st <= c.steps; ++st) {
        const unsigned G = (st == 0 || st == c.steps) ? (Gg > Gl ? Gg : Gl) : Gg;
        k_cdf_step<H><<<G, STEP_NT, 0, s>>>(u, m, st, c.steps, c.batch, c.lr, tb);
    }
    k_cdf_finish<H><<<1, TRAIN_NT, 0, s>>>(m, c.steps, c.knots, c.flags & 1, tb, model);
}

hipError_t train_enqueue(const void* sorted, uint64_t m, int key_bits, const vmps_learned_config& c, float* u,
                         float* tb, vmps_cdf_model* model, hipStream_t s)
{
    if (key_bits == 32)
        k_cdf_features<uint32_t><<<grid1(m), 256, 0, s>>>((const uint32_t*)sorted, m, 32, c.feature_bits, u, model);
    else
        k_cdf_features<uint64_t><<<grid1(m), 256, 0, s>>>((const uint64_t*)sorted, m, 64, c.feature_bits, u, model);
    switch (c.hidden) {
    case 16: train_launches<16>(u, m, c, tb, model, s); break;
    case 32: train_launches<32>(u, m, c, tb, model, s); break;
    default: train_launches<64>(u, m, c, tb, model, s); break;
    }
    return hipGetLastError();
}

hipError_t grad_enqueue(const float* params, int H, const float* u, const float* y, int nb, float* grad, float* loss,
                        hipStream_t s)
{
    switch (H) {
    case 16: k_cdf_grad<16><<<1, TRAIN_NT, 0, s>>>(params, u, y, nb, grad, loss); break;
    case 32: k_cdf_grad<32><<<1, TRAIN_NT, 0, s>>>(params, u, y, nb, grad, loss); break;
    default: k_cdf_grad<64><<<1, TRAIN_NT, 0, s>>>(params, u, y, nb, grad, loss); break;
    }
    return hipGetLastError();
}

hipError_t compile_enqueue(const float* params, int H, uint64_t z_lo, uint64_t z_hi, int key_bits, int fbits, int K,
                           vmps_cdf_model* model, hipStream_t s)
{
    switch (H) {
    case 16: k_cdf_compile<16><<<1, TRAIN_NT, 0, s>>>(params, z_lo, z_hi, key_bits, fbits, K, model); break;
    case 32: k_cdf_compile<32><<<1, TRAIN_NT, 0, s>>>(params, z_lo, z_hi, key_bits, fbits, K, model); break;
    default: k_cdf_compile<64><<<1, TRAIN_NT, 0, s>>>(params, z_lo, z_hi, key_bits, fbits, K, model); break;
    }
    return hipGetLastError();
}

hipError_t bucket_ids_enqueue(const void* keys, uint64_t n, int key_bits, const vmps_cdf_model* model, uint32_t B,
                              uint32_t* ids, hipStream_t s)
{
    const unsigned g = (unsigned)(ceil_div(n ? n : 1, 256) < 8192 ? ceil_div(n ? n : 1, 256) : 8192);
    if (key_bits == 32) k_bucket_ids<uint32_t><<<g, 256, 0, s>>>((const uint32_t*)keys, n, model, B, ids);
    else k_bucket_ids<uint64_t><<<g, 256, 0, s>>>((const uint64_t*)keys, n, model, B, ids);
    return hipGetLastError();
}

hipError_t learned_stats_enqueue(const int64_t* off, uint32_t B, uint32_t T, const vmps_cdf_model* model,
                                 const void* sample, uint64_t m, int key_bits, uint64_t* part,
                                 vmps_learned_stats* st, hipStream_t s)
{
    if (key_bits == 64)
        k_learned_judge<uint64_t><<<JUDGE_GRID, 256, 0, s>>>((const uint64_t*)sample, m, model, B, part);
    else
        k_learned_judge<uint32_t><<<JUDGE_GRID, 256, 0, s>>>((const uint32_t*)sample, m, model, B, part);
    k_learned_stats<<<1, 256, 0, s>>>(off, B, T, model, m, part, st);
    return hipGetLastError();
}

}  // namespace vmps

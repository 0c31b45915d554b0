// Exact enumeration of every Bernoulli path (eq. (f13)) and the
// deterministic reduction of its partial sums (eqs. (f14), (f15)).
//
// Section 3 gives each of M processes the 2^(N-r) paths behind one r-step
// prefix and sums the local values with one reduce; with more partitions than
// processes it assigns them cyclically (partition m to process m mod M).
// Here a workgroup of kWaves waves is the process and its unit of work is a
// rectangle of paths: a chunk of up to kMaxChunk consecutive prefixes of the
// prefix table times kWaves tiles of kTile = 64 kJ suffixes.  Workgroups
// take these rectangles cyclically (g, g + G, g + 2G, ...) from a list
// ordered largest-first, so no counter and no atomics are involved.
// Per rectangle:
//   - the workgroup copies the chunk's prefix records into LDS;
//   - each wave owns one suffix tile and keeps its kJ suffix operands Y_s per
//     lane in VGPRs;
//   - the wave walks the chunk; every prefix record is read from LDS by all
//     lanes at one address (a broadcast), eight records per step;
//   - each path costs one subtraction whose clamp modifier performs the
//     max(., 0) and one add: on a binomial tree every prefix with a ups has
//     the same multiplier c_a and path weight W_a (the price at the prefix's
//     end is S u^(2a - P)), so the prefixes are visited in up-count order,
//     records hold X_z alone, and each group's sums are weighted by W_a c_a
//     once; time-varying and trinomial trees and Shared-Sample draws keep
//     {X_z, c_z} records in natural order and one fused multiply-add;
//   - the lane sum is weighted by the suffix weights omega_s, and the wave
//     sum goes to the partial slot of (option, chunk, tile) in FP64.  The
//     reduction kernel sums each option's partials in a fixed order, so the
//     result does not depend on which workgroup ran which rectangle.
//
// FP32 form, binomial trees: X and Y are FP32, in the same up-count order,
// so a path costs one clamped FP32 subtraction and one FP32 add.  The lane sums each block of kBlock prefixes as a pairwise tree,
// chains kRunBlocks trees into a run, folds each run into a Kahan (sum,
// compensation) pair, and at the group's end adds W_a c_a omega_s (sum -
// comp), in FP64, to one FP64 accumulator.  Each path's term thus passes
// through at most 1 + log2(kBlock) + (kRunBlocks - 1) FP32 roundings before
// the Kahan fold, which is what the result's error bound counts.
//
// FP32 form, time-varying and trinomial trees (no up-count groups) and
// Shared-Sample draws: records {X, g} with g = c / W (the weight folded into
// g for the trees), runs of kKahanRun fused multiply-adds folded by Kahan as
// above.  Weights, the affine part and all reductions stay FP64.
#include "bt_internal.hpp"
#include "bound.hpp"

namespace bt {
namespace {

typedef const __attribute__((address_space(4))) double *cdptr;
typedef const __attribute__((address_space(4))) int64_t *ciptr;
typedef const __attribute__((address_space(4))) OptDev *coptr;
// Device-memory pointers: global loads count against the vector-memory wait
// counter only, where generic (flat) ones also hold up LDS waits.
typedef const __attribute__((address_space(1))) double *gdptr;

// base[i] where ok, else 0.  The load itself is unconditional (element 0,
// which every caller's array has, stands in where !ok), so a lane's loads
// of a loop are all in flight together: a load under a branch whose other
// side writes the same register has to complete before the two paths join,
// which serialises a loop of them into one memory round trip each.
template <typename T, typename PTR>
__device__ __forceinline__ T load_or_zero(PTR base, int64_t i, bool ok)
{
    const T v = base[ok ? i : 0];
    return ok ? v : T(0);
}

// Copies a chunk's n records into LDS (the caller synchronises the
// workgroup afterwards).
template <typename T>
__device__ __forceinline__ void stage_chunk(T *dst, const T *src, int n)
{
    for (int i = (int)threadIdx.x; i < n; i += 64 * kWaves) dst[i] = src[i];
}

template <int SIGN>
__device__ __forceinline__ double cdiff(double y, double x)
{
    const double d = SIGN > 0 ? (y - x) : (x - y);
    return __builtin_fmin(__builtin_fmax(d, 0.0), 1.0);
}

template <int SIGN>
__device__ __forceinline__ float cdiff(float y, float x)
{
    const float d = SIGN > 0 ? (y - x) : (x - y);
    return __builtin_fminf(__builtin_fmaxf(d, 0.0f), 1.0f);
}

// Four prefixes against the lane's kJ suffixes (FP64).
template <int SIGN>
__device__ __forceinline__ void four64(const double2 r0, const double2 r1, const double2 r2,
                                       const double2 r3, const double (&y)[kJ],
                                       double (&acc)[kJ])
{
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        double a = acc[j];
        a = __builtin_fma(r0.y, cdiff<SIGN>(y[j], r0.x), a);
        a = __builtin_fma(r1.y, cdiff<SIGN>(y[j], r1.x), a);
        a = __builtin_fma(r2.y, cdiff<SIGN>(y[j], r2.x), a);
        a = __builtin_fma(r3.y, cdiff<SIGN>(y[j], r3.x), a);
        acc[j] = a;
    }
}

// Prefix records rec[0..n) (LDS) against the lane's suffixes, FP64, eight
// records per step (the reads of the second four overlap the arithmetic of
// the first).
template <int SIGN>
__device__ __forceinline__ void prefixes_f64(const double2 *rec, int n, const double (&y)[kJ],
                                             double (&acc)[kJ])
{
    int z = 0;
    for (; z + 8 <= n; z += 8) {
        four64<SIGN>(rec[z], rec[z + 1], rec[z + 2], rec[z + 3], y, acc);
        four64<SIGN>(rec[z + 4], rec[z + 5], rec[z + 6], rec[z + 7], y, acc);
    }
    for (; z < n; ++z) {
        const double2 r = rec[z];
#pragma unroll
        for (int j = 0; j < kJ; ++j) acc[j] = __builtin_fma(r.y, cdiff<SIGN>(y[j], r.x), acc[j]);
    }
}

// Four prefixes against the lane's kJ suffixes (FP32), added to the run
// (INIT: starting it; the first product g d is then the run itself, the
// same value the fused multiply-add onto 0 gives).
template <int SIGN, bool INIT>
__device__ __forceinline__ void four32(const float2 r0, const float2 r1, const float2 r2,
                                       const float2 r3, const float (&y)[kJ], float (&run)[kJ])
{
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        float r = INIT ? r0.y * cdiff<SIGN>(y[j], r0.x)
                       : __builtin_fmaf(r0.y, cdiff<SIGN>(y[j], r0.x), run[j]);
        r = __builtin_fmaf(r1.y, cdiff<SIGN>(y[j], r1.x), r);
        r = __builtin_fmaf(r2.y, cdiff<SIGN>(y[j], r2.x), r);
        r = __builtin_fmaf(r3.y, cdiff<SIGN>(y[j], r3.x), r);
        run[j] = r;
    }
}

// One run of up to kKahanRun fused multiply-adds from position z of a group
// ending at gend, folded into the Kahan pair (ks, kc) (sum = ks - kc); z
// ends at the run's end.
template <int SIGN>
__device__ __forceinline__ void fma_run_fold(const float2 *rec, int &z, int gend,
                                             const float (&y)[kJ], float (&ks)[kJ],
                                             float (&kc)[kJ])
{
    const int rend = (z + kKahanRun < gend) ? z + kKahanRun : gend;
    float run[kJ];
    if (z + 4 <= rend) {
        four32<SIGN, true>(rec[z], rec[z + 1], rec[z + 2], rec[z + 3], y, run);
        z += 4;
    } else {
#pragma unroll
        for (int j = 0; j < kJ; ++j) run[j] = 0.0f;
    }
    for (; z + 4 <= rend; z += 4)
        four32<SIGN, false>(rec[z], rec[z + 1], rec[z + 2], rec[z + 3], y, run);
    for (; z < rend; ++z) {
        const float2 r = rec[z];
#pragma unroll
        for (int j = 0; j < kJ; ++j) run[j] = __builtin_fmaf(r.y, cdiff<SIGN>(y[j], r.x), run[j]);
    }
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        const float yv = run[j] - kc[j];
        const float t = ks[j] + yv;
        kc[j] = (t - ks[j]) - yv;
        ks[j] = t;
    }
}

// The end of a group in the FP32 {X, g} form: acc[j] += w (ks - kc), FP64.
__device__ __forceinline__ void group_end_f32(double w, const float (&ks)[kJ],
                                              const float (&kc)[kJ], double (&acc)[kJ])
{
#pragma unroll
    for (int j = 0; j < kJ; ++j) acc[j] = __builtin_fma(w, (double)ks[j] - (double)kc[j], acc[j]);
}

// FP32 form over records rec[0..n) of global positions [z0, z0 + n).
template <int SIGN>
__device__ __forceinline__ void prefixes_f32(const float2 *rec, ciptr goff, cdptr Wg, int P,
                                             int64_t z0, int n, const float (&y)[kJ],
                                             double (&acc)[kJ])
{
    int a = 0;
    while (a < P && goff[a + 1] <= z0) ++a;
    int z = 0;
    while (z < n) {
        const int64_t gend64 = goff[a + 1] - z0;
        const int gend = gend64 < n ? (int)gend64 : n;
        float ks[kJ], kc[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) ks[j] = kc[j] = 0.0f;
        while (z < gend) fma_run_fold<SIGN>(rec, z, gend, y, ks, kc);
        group_end_f32(Wg[a], ks, kc, acc);
        ++a;
    }
}

// Rectangle (prefix chunk c, suffix-tile group g) of an option's local
// workgroup item l.  Workgroups go to the 8 XCDs round-robin by index, and
// each XCD has its own L2; with od.xa = a > 0 (a divides the chunk count and
// 8 / a the group count, and the option's items start on a multiple of 8)
// the items of XCD x = l mod 8 form one block of chunks x / (8/a) and groups
// x mod (8/a), so an XCD fetches 1/a of the option's prefix records and a/8
// of its suffix operands instead of all prefixes.  Any order gives the same
// results: a rectangle's partial slot depends on (c, g) alone.
template <typename OD>
__device__ __forceinline__ void rect_of(const OD &od, int64_t l, int64_t &c, int64_t &g)
{
    if (od.xa > 0) {
        const int64_t b = 8 / od.xa;                 // group blocks
        const int64_t cb = od.nchunks / od.xa, gb = od.groups / b;  // block extents
        const int64_t x = l & 7, j = l >> 3;
        const int64_t jc = j / gb;
        c = (x / b) * cb + jc;
        g = (x % b) * gb + (j - jc * gb);
    } else {
        c = l / od.groups;
        g = l - c * od.groups;
    }
}

// FP32 binomial form: one block of kBlock prefix operands x[] against the
// lane's suffixes; each suffix's kBlock clamped differences are summed as a
// balanced tree, which starts the run (INIT) or is added to it.
template <int SIGN, bool INIT>
__device__ __forceinline__ void block_tree(const float (&x)[kBlock], const float (&y)[kJ],
                                           float (&run)[kJ])
{
    static_assert(kBlock == 16, "the tree below sums 16 terms");
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        float d[kBlock];
#pragma unroll
        for (int q = 0; q < kBlock; ++q) d[q] = cdiff<SIGN>(y[j], x[q]);
        const float t0 = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7]));
        const float t1 = ((d[8] + d[9]) + (d[10] + d[11])) + ((d[12] + d[13]) + (d[14] + d[15]));
        run[j] = INIT ? t0 + t1 : run[j] + (t0 + t1);
    }
}

// The kBlock operands from position z; past the group's end (gend) the
// padding value, whose clamped difference is exactly 0.  In a block that
// reaches past gend every record is still read (rec has kBlock entries of
// padding after the chunk) and then selected, so the block takes no branch
// per record.
__device__ __forceinline__ void load_block(const float *rec, int z, int gend, float pad,
                                           float (&x)[kBlock])
{
    if (z + kBlock <= gend) {
#pragma unroll
        for (int q = 0; q < kBlock; ++q) x[q] = rec[z + q];
    } else {
        const int left = gend - z;
#pragma unroll
        for (int q = 0; q < kBlock; ++q) {
            const float v = rec[z + q];  // inside rec's kBlock padding
            x[q] = q < left ? v : pad;
        }
    }
}

// One run from position z of a group ending at gend: up to kRunBlocks
// trees, the first one starting it, folded into the Kahan pair (ks, kc)
// (sum = ks - kc).  z ends at the run's end (at most gend).
template <int SIGN>
__device__ __forceinline__ void run_fold(const float *rec, int &z, int gend, float pad,
                                         const float (&y)[kJ], float (&ks)[kJ], float (&kc)[kJ])
{
    float run[kJ];
    float x[kBlock];
    load_block(rec, z, gend, pad, x);
    block_tree<SIGN, true>(x, y, run);
    z += kBlock;
#pragma unroll 1
    for (int b = 1; b < kRunBlocks && z < gend; ++b, z += kBlock) {
        load_block(rec, z, gend, pad, x);
        block_tree<SIGN, false>(x, y, run);
    }
    if (z > gend) z = gend;
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        const float yv = run[j] - kc[j];
        const float t = ks[j] + yv;
        kc[j] = (t - ks[j]) - yv;
        ks[j] = t;
    }
}

// The lane's suffix weights o[j] = om_lane[64 j], read at an up-count
// group's end (from L2: a few coalesced loads per group) rather than kept in
// 2 kJ VGPRs: om_lane points at the lane's first suffix weight, `left`
// suffixes of the option remain from there (suffix j of the lane exists if
// 64 j < left, else o[j] = 0), and full (uniform over the wave) says that
// every lane has all kJ suffixes, so the loads need no bounds selects.
__device__ __forceinline__ void lane_weights(gdptr om_lane, int left, bool full,
                                             double (&o)[kJ])
{
    // keep the loads and their bounds here, not hoisted out of the caller's
    // loop into VGPRs
    gdptr om = om_lane;
    int nl = left;
    __asm__ volatile("" : "+v"(om), "+v"(nl));
    if (full) {
#pragma unroll
        for (int j = 0; j < kJ; ++j) o[j] = om[64 * j];
    } else {
#pragma unroll
        for (int j = 0; j < kJ; ++j) o[j] = load_or_zero<double>(om, 64 * j, 64 * j < nl);
    }
    // all sixteen loads issued before any is used (otherwise the compiler,
    // short of registers here, waits for each in turn)
    static_assert(kJ == 16, "the register pin below names 16 weights");
    __asm__ volatile("" : "+v"(o[0]), "+v"(o[1]), "+v"(o[2]), "+v"(o[3]), "+v"(o[4]),
                     "+v"(o[5]), "+v"(o[6]), "+v"(o[7]));
    __asm__ volatile("" : "+v"(o[8]), "+v"(o[9]), "+v"(o[10]), "+v"(o[11]), "+v"(o[12]),
                     "+v"(o[13]), "+v"(o[14]), "+v"(o[15]));
}

// Sum over the lane's suffixes of omega_s E_s, the separable part of f
// (om_lane, left, full as in lane_weights; e_lane points at the lane's
// first E_s).  The terms are added in suffix order either way.
__device__ __forceinline__ double sep_sum(gdptr om_lane, gdptr e_lane, int left, bool full)
{
    double sep = 0.0;
    if (full) {
#pragma unroll
        for (int j = 0; j < kJ; ++j) sep = __builtin_fma(om_lane[64 * j], e_lane[64 * j], sep);
    } else {
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            const bool ok = 64 * j < left;
            const double o = load_or_zero<double>(om_lane, 64 * j, ok);
            const double e = load_or_zero<double>(e_lane, 64 * j, ok);
            sep = ok ? __builtin_fma(o, e, sep) : sep;
        }
    }
    return sep;
}

// The end of an up-count group in the FP32 binomial form: adds w omega_s
// (ks - kc) over the lane's suffixes to acc, in FP64 (the weights as in
// lane_weights).
__device__ __forceinline__ void group_end(double w, gdptr om_lane, int left, bool full,
                                          const float (&ks)[kJ], const float (&kc)[kJ],
                                          double &acc)
{
    double o[kJ];
    lane_weights(om_lane, left, full, o);
#pragma unroll
    for (int j = 0; j < kJ; ++j) acc = __builtin_fma(w * o[j], (double)ks[j] - (double)kc[j], acc);
}

// Records rec[0..n) (LDS, global positions [z0, z0 + n)) of an up-count
// ordered FP32 binomial table against the lane's suffixes.  The records of
// up-count group a hold X_z - Cg[a]; at each group's start the lane forms
// its suffix operands Y_s - Cg[a] from the FP64 table (y_lane[64 j], for
// 64 j < left), so both operands of the subtraction are small near the
// money.  A block that reaches past its group's end reads the padding
// value in place of the prefixes beyond it, so every term goes through the
// same tree.  rec must be readable up to index n + kBlock.  Each group
// ends in group_end (om_lane, left as there); full (uniform over the wave)
// says that every lane has all kJ suffixes, so the loads need no bounds
// selects.
template <int SIGN>
__device__ __forceinline__ void prefixes_grouped32(const float *rec, ciptr goff, cdptr Wg,
                                                   cdptr Cg, int P, int64_t z0, int n,
                                                   gdptr y_lane, gdptr om_lane, int left,
                                                   bool full, double &acc)
{
    const float pad = SIGN > 0 ? INFINITY : -INFINITY;
    int a = 0;
    while (a < P && goff[a + 1] <= z0) ++a;
    int z = 0;
    while (z < n) {
        const int64_t gend64 = goff[a + 1] - z0;
        const int gend = gend64 < n ? (int)gend64 : n;
        float y[kJ];
        {
            const double cg = Cg[a];
            gdptr yp = y_lane;
            int nl = left;
            // keep the loads at the group's start, not hoisted into VGPRs
            __asm__ volatile("" : "+v"(yp), "+v"(nl));
            if (full) {
#pragma unroll
                for (int j = 0; j < kJ; ++j) y[j] = (float)(yp[64 * j] - cg);
            } else {
#pragma unroll
                for (int j = 0; j < kJ; ++j) {
                    const bool ok = 64 * j < nl;
                    const double v = load_or_zero<double>(yp, 64 * j, ok);
                    y[j] = ok ? (float)(v - cg) : 0.0f;
                }
            }
        }
        float ks[kJ], kc[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) ks[j] = kc[j] = 0.0f;
        // two runs per iteration, so that the second fold's new sum can take
        // the register the first one read its sum from, and the group's end
        // after each of them, so that neither exit copies the sums
        for (;;) {
            run_fold<SIGN>(rec, z, gend, pad, y, ks, kc);
            if (z >= gend) {
                group_end(Wg[a], om_lane, left, full, ks, kc, acc);
                break;
            }
            run_fold<SIGN>(rec, z, gend, pad, y, ks, kc);
            if (z >= gend) {
                group_end(Wg[a], om_lane, left, full, ks, kc, acc);
                break;
            }
        }
        ++a;
    }
}

// The FP32 binomial kernel: rectangles as in enumerate_kernel, X-only
// records, one FP64 accumulator per lane.  The last nbound workgroups each
// form the error bound's sums over one prefix chunk of the plan (bound.hpp).
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(4))) void enumerate_grouped32_kernel(
    coptr opts, int nopts, int64_t nbitems, double *__restrict__ partial, int64_t nbound)
{
    const int64_t rgrid = (int64_t)gridDim.x - nbound;  // workgroups taking rectangles
    if ((int64_t)blockIdx.x >= rgrid) {
        bound::chunk(opts, nopts, (int64_t)blockIdx.x - rgrid);
        return;
    }
    __shared__ float rec[kMaxChunk + kBlock];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t bi = blockIdx.x; bi < nbitems; bi += rgrid) {
        int lo = 0, hi = nopts - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (opts[mid].bitem_begin <= bi) lo = mid; else hi = mid - 1;
        }
        const auto &od = opts[lo];
        int64_t c, g;
        rect_of(od, bi - od.bitem_begin, c, g);
        const int64_t z0 = c * od.chunk;
        const int n = (int)((z0 + od.chunk < od.npre) ? od.chunk : od.npre - z0);
        __syncthreads();
        stage_chunk(rec, od.XG + z0, n);
        __syncthreads();
        int64_t t = g * kWaves + wave;
        int part = 0;
        if (od.wsplit > 1) {
            t = wave / od.wsplit;
            part = wave - (int)t * od.wsplit;
        }
        if (t >= od.tiles) continue;
        const int per = (n + od.wsplit - 1) / od.wsplit;
        const int zb = part * per < n ? part * per : n;
        const int zn = (zb + per < n ? zb + per : n) - zb;
        const int64_t sbase = t * kTile + lane;
        double acc = 0.0;
        const float *r = rec + zb;
        // suffixes of the option from the lane's first one (<= 2^16)
        const int left = sbase < od.nsuf ? (int)(od.nsuf - sbase) : 0;
        const gdptr y_lane = (gdptr)od.Y + (sbase < od.nsuf ? sbase : 0);
        const gdptr om_lane = (gdptr)od.Om + (sbase < od.nsuf ? sbase : 0);
        const bool full = t * kTile + kTile <= od.nsuf;  // every lane has kJ suffixes
        if (od.sign > 0)
            prefixes_grouped32<1>(r, (ciptr)od.goff, (cdptr)od.Wg, (cdptr)od.Cg, od.P, z0 + zb,
                                  zn, y_lane, om_lane, left, full, acc);
        else
            prefixes_grouped32<-1>(r, (ciptr)od.goff, (cdptr)od.Wg, (cdptr)od.Cg, od.P, z0 + zb,
                                   zn, y_lane, om_lane, left, full, acc);
        // the separable part of the chunk enters once, through part 0 (its
        // loads come after the prefix loop, where they do not compete with
        // the loop's registers; the lane's E pointer is formed here, from
        // its omega pointer, rather than kept through the loop)
        gdptr om_after = om_lane;
        __asm__ volatile("" : "+v"(om_after));
        const gdptr e_lane = (gdptr)od.E + (om_after - (gdptr)od.Om);
        const double sep = sep_sum(om_after, e_lane, left, full);
        const double cu = part == 0 ? ((cdptr)od.chunkU)[c] : 0.0;
        double lt = __builtin_fma(sep, cu, acc);
        for (int off = 32; off >= 1; off >>= 1) lt += __shfl_xor(lt, off);
        if (lane == 0) partial[od.item_begin + (c * od.tiles + t) * od.wsplit + part] = lt;
    }
}

// FP64 form, binomial trees: four prefix operands against the lane's kJ
// suffixes, each clamped difference added to the suffix's group sum.
template <int SIGN>
__device__ __forceinline__ void four_add64(const double x0, const double x1, const double x2,
                                           const double x3, const double (&y)[kJ],
                                           double (&sg)[kJ])
{
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        double t = sg[j];
        t += cdiff<SIGN>(y[j], x0);
        t += cdiff<SIGN>(y[j], x1);
        t += cdiff<SIGN>(y[j], x2);
        t += cdiff<SIGN>(y[j], x3);
        sg[j] = t;
    }
}

// Records rec[0..n) (LDS, global positions [z0, z0 + n)) of an up-count
// ordered FP64 binomial table against the lane's suffix operands y[].  All
// prefixes of up-count group a share the multiplier c_a and the weight
// W_a, so a path costs one clamped subtraction and one plain add into the
// group sums sg[j]; at the group's end they fold into the lane's
// accumulator as acc += Wg[a] sum_j omega_j sg[j], with the sixteen suffix
// weights read from L2 together (om_lane[64 j] for 64 j < left).
template <int SIGN>
__device__ __forceinline__ void prefixes_grouped64(const double *rec, ciptr goff, cdptr Wg,
                                                   int P, int64_t z0, int n,
                                                   const double (&y)[kJ], gdptr om_lane,
                                                   int left, double &acc)
{
    int a = 0;
    while (a < P && goff[a + 1] <= z0) ++a;
    int z = 0;
    while (z < n) {
        const int64_t gend64 = goff[a + 1] - z0;
        const int gend = gend64 < n ? (int)gend64 : n;
        double sg[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) sg[j] = 0.0;
        for (; z + 8 <= gend; z += 8) {
            four_add64<SIGN>(rec[z], rec[z + 1], rec[z + 2], rec[z + 3], y, sg);
            four_add64<SIGN>(rec[z + 4], rec[z + 5], rec[z + 6], rec[z + 7], y, sg);
        }
        for (; z < gend; ++z) {
            const double x = rec[z];
#pragma unroll
            for (int j = 0; j < kJ; ++j) sg[j] += cdiff<SIGN>(y[j], x);
        }
        // (with the bounds selects even on full tiles: the unselected
        // loads' addresses take registers that four waves per SIMD leave
        // this kernel no room for)
        double o[kJ];
        lane_weights(om_lane, left, false, o);
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kJ; ++j) t = __builtin_fma(o[j], sg[j], t);
        acc = __builtin_fma(Wg[a], t, acc);
        ++a;
    }
}

// The FP64 binomial kernel: rectangles as in enumerate_kernel, X-only
// records in up-count order, one FP64 accumulator per lane.
__global__ __launch_bounds__(64 * kWaves) void enumerate_grouped64_kernel(
    coptr opts, int nopts, int64_t nbitems, double *__restrict__ partial)
{
    __shared__ double rec[kMaxChunk];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t bi = blockIdx.x; bi < nbitems; bi += gridDim.x) {
        int lo = 0, hi = nopts - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (opts[mid].bitem_begin <= bi) lo = mid; else hi = mid - 1;
        }
        const auto &od = opts[lo];
        int64_t c, g;
        rect_of(od, bi - od.bitem_begin, c, g);
        const int64_t z0 = c * od.chunk;
        const int n = (int)((z0 + od.chunk < od.npre) ? od.chunk : od.npre - z0);
        __syncthreads();
        stage_chunk(rec, od.XC + z0, n);
        __syncthreads();
        int64_t t = g * kWaves + wave;
        int part = 0;
        if (od.wsplit > 1) {
            t = wave / od.wsplit;
            part = wave - (int)t * od.wsplit;
        }
        if (t >= od.tiles) continue;
        const int per = (n + od.wsplit - 1) / od.wsplit;
        const int zb = part * per < n ? part * per : n;
        const int zn = (zb + per < n ? zb + per : n) - zb;
        const int64_t sbase = t * kTile + lane;
        const bool full = t * kTile + kTile <= od.nsuf;  // every lane has kJ suffixes
        double y[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            const int64_t s = sbase + 64 * j;
            y[j] = load_or_zero<double>(od.Y, s, s < od.nsuf);
        }
        // suffixes of the option from the lane's first one (<= 2^16)
        const int left = sbase < od.nsuf ? (int)(od.nsuf - sbase) : 0;
        const gdptr om_lane = (gdptr)od.Om + (sbase < od.nsuf ? sbase : 0);
        const gdptr e_lane = (gdptr)od.E + (sbase < od.nsuf ? sbase : 0);
        double acc = 0.0;
        if (od.sign > 0)
            prefixes_grouped64<1>(rec + zb, (ciptr)od.goff, (cdptr)od.Wg, od.P, z0 + zb, zn, y,
                                  om_lane, left, acc);
        else
            prefixes_grouped64<-1>(rec + zb, (ciptr)od.goff, (cdptr)od.Wg, od.P, z0 + zb, zn, y,
                                   om_lane, left, acc);
        // the separable part of the chunk enters once, through part 0
        const double sep = sep_sum(om_lane, e_lane, left, full);
        const double cu = part == 0 ? ((cdptr)od.chunkU)[c] : 0.0;
        double lt = __builtin_fma(sep, cu, acc);
        for (int off = 32; off >= 1; off >>= 1) lt += __shfl_xor(lt, off);
        if (lane == 0) partial[od.item_begin + (c * od.tiles + t) * od.wsplit + part] = lt;
    }
}

template <bool F32>
struct Rec {
    typedef double2 type;
};
template <>
struct Rec<true> {
    typedef float2 type;
};

// The FP32 form asks for four waves per SIMD (at most 128 VGPRs): the
// fourth wave hides more of the LDS and Kahan-fold latency.  The FP64 form
// reaches four waves unforced.
template <bool F32>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(F32 ? 4 : 1))) void enumerate_kernel(coptr opts, int nopts,
                                                                int64_t nbitems,
                                                                double *__restrict__ partial)
{
    typedef typename Rec<F32>::type R;
    __shared__ R rec[kMaxChunk];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t bi = blockIdx.x; bi < nbitems; bi += gridDim.x) {
        // Option owning this workgroup item: last one with bitem_begin <= bi.
        int lo = 0, hi = nopts - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (opts[mid].bitem_begin <= bi) lo = mid; else hi = mid - 1;
        }
        const auto &od = opts[lo];
        int64_t c, g;
        rect_of(od, bi - od.bitem_begin, c, g);
        const int64_t z0 = c * od.chunk;
        const int n = (int)((z0 + od.chunk < od.npre) ? od.chunk : od.npre - z0);
        // Stage the chunk's prefix records in LDS.
        __syncthreads();
        if constexpr (F32)
            stage_chunk(rec, reinterpret_cast<const R *>(od.XG) + z0, n);
        else
            stage_chunk(rec, reinterpret_cast<const R *>(od.XC) + z0, n);
        __syncthreads();
        // Tile of this wave; with fewer tiles than waves (wsplit > 1, one
        // group) wsplit waves share a tile, each taking a part of the chunk.
        int64_t t = g * kWaves + wave;
        int part = 0;
        if (od.wsplit > 1) {
            t = wave / od.wsplit;
            part = wave - (int)t * od.wsplit;
        }
        if (t >= od.tiles) continue;
        const int per = (n + od.wsplit - 1) / od.wsplit;
        const int zb = part * per < n ? part * per : n;
        const int zn = (zb + per < n ? zb + per : n) - zb;
        const int64_t sbase = t * kTile + lane;
        const bool full = t * kTile + kTile <= od.nsuf;  // every lane has kJ suffixes: no selects
        double acc[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) acc[j] = 0.0;
        if constexpr (F32) {
            float y[kJ];
            if (full) {
#pragma unroll
                for (int j = 0; j < kJ; ++j) y[j] = od.Y32[sbase + 64 * j];
            } else {
#pragma unroll
                for (int j = 0; j < kJ; ++j) {
                    const int64_t s = sbase + 64 * j;
                    y[j] = load_or_zero<float>(od.Y32, s, s < od.nsuf);
                }
            }
            const float2 *r = reinterpret_cast<const float2 *>(rec);
            if (od.sign > 0)
                prefixes_f32<1>(r + zb, (ciptr)od.goff, (cdptr)od.Wg, od.P, z0 + zb, zn, y, acc);
            else
                prefixes_f32<-1>(r + zb, (ciptr)od.goff, (cdptr)od.Wg, od.P, z0 + zb, zn, y, acc);
        } else {
            double y[kJ];
            if (full) {
#pragma unroll
                for (int j = 0; j < kJ; ++j) y[j] = od.Y[sbase + 64 * j];
            } else {
#pragma unroll
                for (int j = 0; j < kJ; ++j) {
                    const int64_t s = sbase + 64 * j;
                    y[j] = load_or_zero<double>(od.Y, s, s < od.nsuf);
                }
            }
            const double2 *r = reinterpret_cast<const double2 *>(rec);
            if (od.sign > 0)
                prefixes_f64<1>(r + zb, zn, y, acc);
            else
                prefixes_f64<-1>(r + zb, zn, y, acc);
        }
        // the separable part of the chunk enters once, through part 0
        const double cu = part == 0 ? ((cdptr)od.chunkU)[c] : 0.0;
        if (od.persuf) {
            // Shared-Sample MC: keep each drawn suffix's sum over the part.
            double *row = od.persuf + (c * od.wsplit + part) * od.nsuf;
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const int64_t s = sbase + 64 * j;
                if (s < od.nsuf) row[s] = __builtin_fma(od.E[s], cu, acc[j]);
            }
            continue;
        }
        double lt = 0.0;
        if (full) {
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const int64_t s = sbase + 64 * j;
                lt = __builtin_fma(od.Om[s], __builtin_fma(od.E[s], cu, acc[j]), lt);
            }
        } else {
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const int64_t s = sbase + 64 * j;
                const bool ok = s < od.nsuf;
                const double o = load_or_zero<double>(od.Om, s, ok);
                const double e = load_or_zero<double>(od.E, s, ok);
                lt = ok ? __builtin_fma(o, __builtin_fma(e, cu, acc[j]), lt) : lt;
            }
        }
        for (int off = 32; off >= 1; off >>= 1) lt += __shfl_xor(lt, off);
        if (lane == 0) partial[od.item_begin + (c * od.tiles + t) * od.wsplit + part] = lt;
    }
}

__global__ void reset_counter_kernel(unsigned long long *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

// One workgroup per option: thread t sums partial[begin + t + kReduceThreads i]
// in order, then a fixed tree over the threads; the total times e^{-rT} is
// the option's value.  The order depends only on the item count.
//
// Error bound (plans with bound sums): the table kernel bounded the rounding
// error of every stored X_z, U_z, Y_s, E_s; since max(., 0) is 1-Lipschitz,
// the value moves by at most
//     e^{-rT} [ sum_z c_z rhoX_z sum_s om_s + sum_z c_z sum_s om_s rhoY_s
//              + sum_z W_z rhoU_z sum_s om_s |E_s| + sum_z W_z |U_z| sum_s om_s rhoE_s ]
// through them (the FP32 binomial form replaces the first two sums by the
// bound kernel's sum over the paths that can reach the money); every other
// rounding (weights, the clamped subtraction, the FP32 or FP64 sums, the
// reduction, the discount) is relative to a sum of nonnegative terms, hence
// at most eps_rel times the value.  A factor 1 + 2^-20 covers the
// second-order terms of both parts.
constexpr int kReduceThreads = 256;
constexpr int kRw = kReduceThreads / 64;

__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(
    const OptDev *__restrict__ opts, int nopts, const double *__restrict__ partial,
    double *__restrict__ values)
{
    __shared__ double red[9][kRw];
    const OptDev &od = opts[blockIdx.x];
    warm_scalar_cache(od);
    const int tid = threadIdx.x;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // (unrolled so that the loads of several steps are in flight together;
    // each thread still adds its values in index order)
    const gdptr part = (gdptr)partial + od.item_begin;
#pragma unroll 8
    for (int64_t i = tid; i < od.nitems; i += kReduceThreads) v[0] += part[i];
    const bool bound = od.bnd_pre != nullptr;
    if (bound) {
        const gdptr pre = (gdptr)od.bnd_pre, cu = (gdptr)od.chunkU, suf = (gdptr)od.bnd_suf;
        for (int64_t c = tid; c < od.nchunks; c += kReduceThreads) {
            v[1] += pre[4 * c];      // sum c rhoX
            v[2] += pre[4 * c + 1];  // sum c
            v[3] += pre[4 * c + 2];  // sum W rhoU
            v[4] += cu[c];           // sum W U
        }
        for (int64_t j = tid; j < od.nsufjobs; j += kReduceThreads) {
            v[5] += suf[4 * j];      // sum om rhoY
            v[6] += suf[4 * j + 1];  // sum om |E|
            v[7] += suf[4 * j + 2];  // sum om rhoE
            v[8] += suf[4 * j + 3];  // sum om
        }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_xor(v[q], off);
        if ((tid & 63) == 0) red[q][tid >> 6] = v[q];
    }
    __syncthreads();
    if (tid == 0) {
        double t[9];
        for (int q = 0; q < 9; ++q) {
            t[q] = 0.0;
            for (int w = 0; w < kRw; ++w) t[q] += red[q][w];
        }
        const double value = od.disc * t[0];
        values[od.out_index] = value;
        if (bound) {
            // FP32 binomial form: the bound kernel's sums over the paths
            // that can reach the money, in place of the sums over all paths
            const double xy = od.hist ? t[1] : t[1] * t[8] + t[2] * t[5];
            const double in = xy + t[3] * t[6] + t[4] * t[7];
            values[nopts + od.out_index] =
                (od.disc * in + od.eps_rel * fabs(value)) * (1.0 + 0x1p-20);
        }
    }
}

}  // namespace

hipError_t launch_reset_counter(unsigned long long *d_counter, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, d_counter);
    return hipGetLastError();
}

hipError_t launch_enumerate(const OptDev *d_opts, int nopts, int64_t nbitems,
                            double *d_partial, int mode, int grid, int64_t bound_chunks,
                            hipStream_t s)
{
    if (nopts <= 0 || nbitems <= 0) return hipSuccess;
    const dim3 block(64 * kWaves);
    if (mode == 2)
        hipLaunchKernelGGL(enumerate_grouped32_kernel, dim3((unsigned)(grid + bound_chunks)), block,
                           0, s, (coptr)d_opts, nopts, nbitems, d_partial, bound_chunks);
    else if (mode == 3)
        hipLaunchKernelGGL(enumerate_grouped64_kernel, dim3(grid), block, 0, s, (coptr)d_opts,
                           nopts, nbitems, d_partial);
    else if (mode == 1)
        hipLaunchKernelGGL(enumerate_kernel<true>, dim3(grid), block, 0, s, (coptr)d_opts, nopts,
                           nbitems, d_partial);
    else
        hipLaunchKernelGGL(enumerate_kernel<false>, dim3(grid), block, 0, s, (coptr)d_opts, nopts,
                           nbitems, d_partial);
    return hipGetLastError();
}

int enumerate_max_blocks_per_cu(int mode)
{
    int nb = 0;
    hipError_t e;
    if (mode == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(enumerate_grouped32_kernel), 64 * kWaves, 0);
    else if (mode == 3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(enumerate_grouped64_kernel), 64 * kWaves, 0);
    else if (mode == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(enumerate_kernel<true>), 64 * kWaves, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(enumerate_kernel<false>), 64 * kWaves, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_reduce(const OptDev *d_opts, int nopts,
                         const double *d_partial, double *d_values,
                         hipStream_t s)
{
    if (nopts <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(nopts), dim3(kReduceThreads), 0, s, d_opts, nopts,
                       d_partial, d_values);
    return hipGetLastError();
}

}  // namespace bt

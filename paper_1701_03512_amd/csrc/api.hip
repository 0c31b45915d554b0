// Host side of libbt: argument checking, tree parameters, plans (table
// layout, work list, launch shape), the one-shot pricing calls, graphs and
// the autotuner.  Every number of the method is computed by the kernels; the
// host only sizes, orders and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bt.h"
#include "bt_internal.hpp"
#include "host_common.hpp"

using namespace bt;

// ------------------------------------------------------------------ errors

extern "C" const char *bt_strerror(int code)
{
    switch (code) {
    case BT_OK: return "ok";
    case BT_EINVAL: return "invalid argument";
    case BT_ERANGE: return "size out of supported range";
    case BT_ENOMEM: return "out of memory / over budget";
    case BT_EDEVICE: return "HIP device error or no gfx950 device";
    case BT_EAGAIN: return "not ready";
    case BT_ENOTFOUND: return "unknown ticket";
    case BT_ESHUTDOWN: return "server stopped";
    default: return "unknown error";
    }
}

// ------------------------------------------------------------------ device

namespace bt {

static std::mutex g_dev_mu;
static DeviceInfo g_dev[kMaxDevices];

int ensure_device(DeviceInfo **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BT_EDEVICE;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceInfo &d = g_dev[dev];
    if (!d.ready) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return BT_EDEVICE;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BT_EDEVICE;
        d.device = dev;
        d.cus = prop.multiProcessorCount;
        // a failed lookup only disables bt_price_batch_noalloc (BT_EDEVICE)
        (void)noalloc_attach(&d);
        d.ready = true;
    }
    if (out) *out = &d;
    return BT_OK;
}

int hip_err(hipError_t e) { return e == hipSuccess ? BT_OK : BT_EDEVICE; }

}  // namespace bt

extern "C" int bt_init(int device)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return BT_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return BT_EDEVICE;
    return ensure_device(nullptr);
}

// ------------------------------------------------------------------ params

extern "C" int bt_params(double sigma, double r, double T, int32_t N, int32_t scheme,
                         double *u_out, double *p_out)
{
    if (!(sigma > 0) || !(T > 0) || N < 1 || !u_out || !p_out || !std::isfinite(r))
        return BT_EINVAL;
    const double dt = T / (double)N;
    double u;
    if (scheme == BT_SCHEME_CRR) {
        u = std::exp(sigma * std::sqrt(dt));
    } else if (scheme == BT_SCHEME_SEYDEL) {
        const double beta = 0.5 * (std::exp(-r * dt) + std::exp((r + sigma * sigma) * dt));
        u = beta + std::sqrt(beta * beta - 1.0);
    } else {
        return BT_EINVAL;
    }
    const double d = 1.0 / u;
    const double p = (std::exp(r * dt) - d) / (u - d);
    if (!(p > 0.0 && p < 1.0) || !(u > 1.0)) return BT_EINVAL;
    *u_out = u;
    *p_out = p;
    return BT_OK;
}

// Trinomial step (Boyle's three-jump lattice): u = e^{lambda sigma sqrt(dt)};
// with M = e^{r dt} and V = M^2 (e^{sigma^2 dt} - 1) the up and down
// probabilities that match the mean M and the variance V of the step are
//   p_up   = ((V + M^2 - M) u - (M - 1)) / ((u - 1)(u^2 - 1)),
//   p_down = ((V + M^2 - M) u^2 - (M - 1) u^3) / ((u - 1)(u^2 - 1)).
extern "C" int bt_params_trinomial(double sigma, double r, double T, int32_t N, double lambda,
                                   double *u_out, double *pu_out, double *pd_out)
{
    if (!(sigma > 0) || !(T > 0) || N < 1 || !(lambda > 0) || !std::isfinite(r) || !u_out ||
        !pu_out || !pd_out)
        return BT_EINVAL;
    const double dt = T / (double)N;
    const double u = std::exp(lambda * sigma * std::sqrt(dt));
    const double M = std::exp(r * dt);
    const double V = M * M * (std::exp(sigma * sigma * dt) - 1.0);
    const double den = (u - 1.0) * (u * u - 1.0);
    const double pu = ((V + M * M - M) * u - (M - 1.0)) / den;
    const double pd = ((V + M * M - M) * u * u - (M - 1.0) * u * u * u) / den;
    if (!(u > 1.0) || !(pu > 0.0) || !(pd > 0.0) || !(pu + pd < 1.0)) return BT_EINVAL;
    *u_out = u;
    *pu_out = pu;
    *pd_out = pd;
    return BT_OK;
}

namespace bt {

int check_option(const bt_option *o, int max_n)
{
    if (!o) return BT_EINVAL;
    if (!(o->S > 0) || !(o->u > 1.0) || !(o->p > 0.0 && o->p < 1.0) || !(o->T > 0) ||
        !(o->K >= 0) || !std::isfinite(o->r) || !std::isfinite(o->S) ||
        !std::isfinite(o->u) || !std::isfinite(o->K) || !std::isfinite(o->T))
        return BT_EINVAL;
    if (o->payoff < 0 || o->payoff >= NPAYOFF) return BT_EINVAL;
    if (o->N < 1) return BT_EINVAL;
    if (o->N > max_n) return BT_ERANGE;
    return BT_OK;
}

// ------------------------------------------------------------------ tuning

static std::mutex g_tune_mu;
static bt_tuning g_tuned[2][kExactMaxN + 1];  // zero = not tuned

// Built-in launch shape (before autotuning): lanes own the last k steps,
// k ~ N/2 kept in [10, 16] (all of N for small trees), which balances the
// prefix and suffix tables; chunks of about 2^P / 32 prefixes (FP64) or
// 2^P / 64 (FP32), at least 1024 (or all 2^P prefixes when fewer) and at
// most kMaxChunk; one workgroup per rectangle (the hardware dispatcher
// balances the load).  Measured on MI355X: at N = 32, k = 16 with
// 2048-prefix chunks keeps the FP64 enumeration above 90% of the VALU issue
// rate; in a batch of 4096 trees of depth 16..30, chunks below 1024 cost
// the FP32 form 17% (many short Kahan runs and rectangles).
bt_tuning default_tuning(int N, int precision)
{
    bt_tuning t{};
    t.k = (N <= 10) ? N : std::min(16, std::max(10, (N + 1) / 2));
    const int64_t npre = (int64_t)1 << (N - t.k);
    const int64_t div = (precision == BT_FP32_KAHAN) ? 64 : 32;
    const int64_t chunk = std::min<int64_t>(kMaxChunk, std::max<int64_t>(1024, npre / div));
    t.chunk = (int32_t)chunk;
    t.waves = kWaves;
    t.grid = 0;
    return t;
}

// Launch shape for one tree at a time (the server's exact requests): up to
// N = 31 it spreads a single tree over enough rectangles to occupy the GPU,
// from a search of k = 8..16 x chunks 64..2048 per depth on MI355X (tables
// + enumeration + reduction of one tree; N = 24: 22 us against 88 us with
// the built-in shape).  k stays at least 10, so that a wave's 1024-suffix
// tile is full.  These small rectangles are not the default: in a batch of
// 4096 trees of depth 16..30 they cost 14% (FP64) to 40% (FP32) of the
// built-in shape's throughput.  From N = 32 the built-in shape applies.
bt_tuning one_tree_tuning(int N, int precision)
{
    const bool f32 = precision == BT_FP32_KAHAN;
    bt_tuning t = default_tuning(N, precision);
    if (N <= 10 || N >= 32) return t;
    if (N <= 25) {
        t.k = 10;
        t.chunk = 128;
    } else if (N <= 27) {
        t.k = 10;
        t.chunk = 256;
    } else if (N == 28) {
        t.k = 10;
        t.chunk = f32 ? 256 : 512;
    } else if (N == 29) {
        t.k = 11;
        t.chunk = 512;
    } else {
        t.k = 16;
        t.chunk = 512;
    }
    return t;
}

bt_tuning resolve_tuning(int N, int precision, const bt_tuning *user, bool one_tree,
                         const bt_tuning *depth_table)
{
    bt_tuning t = one_tree ? one_tree_tuning(N, precision) : default_tuning(N, precision);
    if (!one_tree) {
        bt_tuning a;
        if (depth_table) {
            a = depth_table[N];
        } else {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            a = g_tuned[precision ? 1 : 0][N];
        }
        if (a.k) t.k = a.k;
        if (a.chunk) t.chunk = a.chunk;
        if (a.waves) t.waves = a.waves;
    }
    if (user) {
        if (user->k) t.k = user->k;
        if (user->chunk) t.chunk = user->chunk;
        if (user->waves) t.waves = user->waves;
        if (user->grid) t.grid = user->grid;
    }
    if (t.k > N) t.k = N;
    return t;
}

// k larger than an option's N is clamped to N (a batch mixes depths).
int check_tuning(const bt_tuning *t)
{
    if (!t) return BT_OK;
    if (t->k && (t->k < 1 || t->k > 16)) return BT_EINVAL;
    if (t->chunk && (t->chunk < 4 || t->chunk % 4 || t->chunk > kMaxChunk)) return BT_EINVAL;
    if (t->waves && t->waves != kWaves) return BT_EINVAL;
    if (t->grid < 0) return BT_EINVAL;
    return BT_OK;
}

}  // namespace bt

extern "C" int bt_tuning_for(int32_t N, int32_t precision, bt_tuning *out)
{
    if (!out || N < 1 || N > kExactMaxN || (precision != BT_FP64 && precision != BT_FP32_KAHAN))
        return BT_EINVAL;
    *out = resolve_tuning(N, precision, nullptr);
    return BT_OK;
}

// ------------------------------------------------------------------ plans

struct bt_plan {
    int device = -1;
    int precision = 0;
    int n = 0;
    std::vector<OptDev> od;      // LPT order
    std::vector<int32_t> status; // per original index
    std::vector<TableJob> jobs;
    std::vector<bt_tuning> tune; // per original index
    OptDev *d_od = nullptr;
    TableJob *d_jobs = nullptr;
    char *mem = nullptr;
    bool owns_memory = false;
    std::vector<std::vector<int64_t>> host_goff;
    std::vector<double> host_tv;  // per-step u, p uploaded to the plan
    int64_t table_entries = 0;    // sum of the table jobs' entry counts
    double *d_partial = nullptr;
    unsigned long long *d_counter = nullptr;
    double *d_values = nullptr;
    int64_t nitems = 0, nbitems = 0;
    int64_t bound_chunks = 0;  // FP32 binomial plans with a bound: prefix chunks
    int grid = 0, waves = kWaves;
    int mode = 0;        // enumeration kernel (PlanLayout::mode)
    bool bounds = false; // the reduction writes an error bound per option
    bt_tuning used{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};

namespace bt {
// Shared-Sample plan: combine the per-(chunk, draw) partials into
// {value, var_est, var_unbiased} at d_out3 (enqueue).
int plan_shared_combine(bt_plan *pl, double *d_out3, hipStream_t s)
{
    if (!pl || pl->n != 1 || !pl->od[0].persuf) return BT_EINVAL;
    const OptDev &d = pl->od[0];
    return hip_err(launch_shared_combine(d.persuf, (int64_t)d.nchunks * d.wsplit, d.nsuf, d.disc,
                                         d_out3, s));
}
}  // namespace bt

namespace bt {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static int64_t job_entries(const std::vector<TableJob> &jobs)
{
    int64_t e = 0;
    for (const TableJob &j : jobs) e += j.kind == TAB_WEIGHTS ? 1 : j.count;
    return e;
}
static int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

static double pow_int(double b, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// Power-of-two scale so that |X - Y| * 2^-e <= 1 for every prefix and
// suffix of the option (bounds from the tree's extreme paths).
static int scale_exponent(const bt_option &o, int P, int k, double center)
{
    const double uP = pow_int(o.u, P), uk = pow_int(o.u, k);
    double B;
    switch (o.payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT: {
        const double tau = (o.N * o.K + P * o.S * uP) * uP / o.S;
        B = tau + center + k * uk + center;
        break;
    }
    case LOOKBACK_FLOAT: B = uP * uP + uk; break;
    case LOOKBACK_FIXED_PUT: B = o.K * uP / o.S + o.u; break;
    default: B = o.K * uP / o.S + uk; break;
    }
    if (!(B >= 1.0)) return 0;
    int ex = 0;
    std::frexp(B, &ex);  // B < 2^ex
    return ex;
}

static int sign_of(int payoff)
{
    return (payoff == ASIAN_CALL || payoff == EURO_CALL) ? 1 : -1;
}

// X of the prefix whose steps are `first` moves of one kind (up if up_first)
// followed by the rest, with a ups out of P (constant moves), as the table
// kernel's prefix map forms it.
static double prefix_x_of_path(const bt_option &o, int P, int a, bool up_first)
{
    double A = 0.0, M = -INFINITY, m = INFINITY;
    int lev = 0;
    for (int t = 1; t <= P; ++t) {
        const bool up = up_first ? t <= a : t > P - a;
        lev += up ? 1 : -1;
        const double St = o.S * std::pow(o.u, (double)lev);
        A += St;
        M = std::max(M, St);
        m = std::min(m, St);
    }
    const double Pz = P == 0 ? o.S : o.S * std::pow(o.u, (double)lev);
    switch (o.payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT: return (o.N * o.K - A) / Pz;
    case LOOKBACK_FLOAT: return P == 0 ? 0.0 : M / Pz;
    case LOOKBACK_FIXED_PUT: {
        const double kap = o.K / Pz;
        return kap - (P == 0 ? 0.0 : std::max(kap - m / Pz, 0.0));
    }
    default: return o.K / Pz;
    }
}

// Centre of up-count group a of the FP32 binomial form: the midpoint of X
// over the group's two extreme paths (all ups first, all ups last), centred
// and scaled as the tables store X.  Any centre gives the same value; one
// near the group's X keeps the FP32 operands, and their rounding, small.
static double group_centre(const bt_option &o, const OptDev &d, int a)
{
    const double x1 = prefix_x_of_path(o, d.P, a, true);
    const double x2 = prefix_x_of_path(o, d.P, a, false);
    return (0.5 * (x1 + x2) - d.center) * d.inv_scale;
}

// XCD blocking of an option's rectangles (see rect_of in enumerate.hip): the
// number a of chunk blocks (with 8 / a tile-group blocks) that minimises the
// L2 fills over the 8 XCDs, 8/a x the prefix bytes + a x the suffix bytes,
// among the splits the option's shape allows (a divides the chunk count,
// 8 / a the group count, items start on a multiple of 8, one wave part per
// tile); 0 keeps the natural order, whose fills are 8 x the prefix bytes +
// the suffix bytes.
static int32_t xcd_blocking(const OptDev &d, int mode, int64_t bitem_begin)
{
    if (bitem_begin % 8 != 0 || d.nbitems % 8 != 0 || d.wsplit != 1) return 0;
    // bytes a workgroup reads per prefix and per suffix
    const double pre = mode == 2 ? 4.0 : (mode == 1 || mode == 3) ? 8.0 : 16.0;
    const double suf = mode == 2 ? 16.0 : mode == 1 ? 12.0 : 24.0;
    int32_t best = 0;
    double best_cost = 8.0 * pre * d.npre + suf * d.nsuf;  // natural order
    for (int a = 1; a <= 8; a *= 2) {
        const int b = 8 / a;
        if (d.nchunks % a != 0 || d.groups % b != 0) continue;
        const double cost = (8.0 / a) * pre * d.npre + a * suf * d.nsuf;
        if (cost < best_cost) {
            best_cost = cost;
            best = a;
        }
    }
    return best;
}

// Histogram range of v = sign Y_s (centred, scaled) for the FP32 binomial
// bound, from the suffixes' extreme paths; values that round outside fall
// in the end bins.  hw = bins per unit of v.
static void suffix_v_range(const bt_option &o, const OptDev &d, double *vlo, double *hw)
{
    const int k = d.k;
    const double u = o.u;
    double ylo, yhi;
    switch (o.payoff) {
    case ASIAN_CALL:
    case ASIAN_PUT:
        ylo = yhi = 0.0;
        for (int j = 1; j <= k; ++j) {
            ylo += std::pow(u, (double)-j);
            yhi += std::pow(u, (double)j);
        }
        break;
    case LOOKBACK_FLOAT: ylo = 1.0 / u; yhi = std::pow(u, (double)k); break;
    case LOOKBACK_FIXED_PUT: ylo = std::pow(u, (double)-k); yhi = u; break;
    default: ylo = std::pow(u, (double)-k); yhi = std::pow(u, (double)k); break;
    }
    double a = d.sign * (ylo - d.center) * d.inv_scale, b = d.sign * (yhi - d.center) * d.inv_scale;
    if (a > b) std::swap(a, b);
    *vlo = a;
    *hw = b > a ? kHistBins / (b - a) : 0.0;
}

// Bound on the FP64 error of every stored suffix operand Y_s (centred and
// scaled): the table kernel's per-suffix bound (multipliers within eps_suf,
// k - 1 adds, the centring) at the largest operand, k u^k.
static double suffix_y_error(const OptDev &d, double u)
{
    const double ymax = d.k * std::pow(u, (double)d.k);
    return ((d.eps_suf + (d.k + 2) * 0x1p-53) * ymax + 0x1p-53 * (ymax + d.center)) *
           d.inv_scale * (1.0 + 0x1p-20);
}

}  // namespace bt

extern "C" int bt_plan_destroy(bt_plan *plan)
{
    if (!plan) return BT_EINVAL;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (plan->device >= 0 && plan->device != cur) (void)hipSetDevice(plan->device);
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->owns_memory && plan->mem) (void)hipFree(plan->mem);
    if (plan->device >= 0 && plan->device != cur && cur >= 0) (void)hipSetDevice(cur);
    delete plan;
    return BT_OK;
}

namespace bt {

// Shapes of every option of a plan and the byte layout of its device memory:
//   [per-option tables | partials | counter | values | OptDev[] | TableJob[] ]
struct TableOffsets {
    size_t X = 0, Y = 0, Om = 0, E = 0, Y32 = 0, CU = 0, Wg = 0, G = 0, PS = 0, TV = 0, BP = 0,
           BS = 0, HS = 0, end = 0;
};


struct PlanLayout {
    std::vector<OptDev> od;         // original order, table pointers unset
    std::vector<TableOffsets> toff; // byte offsets of each option's tables
    std::vector<bt_tuning> tune;
    std::vector<int> order;         // LPT order -> original index
    std::vector<TableJob> jobs;     // opt = LPT position
    std::vector<std::vector<int64_t>> goff;
    std::vector<size_t> table_off;  // per option, bytes from the start
    int64_t nitems = 0, nbitems = 0, nchunks = 0;
    size_t off_partial = 0, off_counter = 0, off_values = 0, off_od = 0, off_jobs = 0;
    size_t total = 0;
    bool shared = false;
    bool tv = false;
    int mode = 0;  // enumeration kernel: 0 FP64 {X, c}, 1 FP32 {X, g}, 2 FP32 X-only,
                   // 3 FP64 X-only (2 and 3: binomial exact trees, up-count order)
    std::vector<double> tv_host;  // u_1..u_N, p_1..p_N, shared by the options
};

// Suffix-table job size: 256 where every step divides or draws
// (time-varying moves, base-3 digits, Philox suffixes), so that those
// blocks do not become the launch's long pole; for the plain binomial
// tables (a table lookup per step) 2048, or 4096 where each job also
// builds a value histogram for the error bound (xonly), which the bound
// sums read once per job.
static int64_t suffix_job_size(bool tv, bool tri, bool shared, bool xonly)
{
    return (tv || tri || shared) ? 256 : (xonly ? 4096 : 2048);
}

// Relative rounding error of a product of `steps` step probabilities: each
// factor is exact (p_t) or formed with one subtraction (1 - p_t), or two for
// the trinomial middle move 1 - p - pd, relative error (1 + (1 - p)/pm) u.
static double weight_rel_err(int steps, bool tri, double p, double pd)
{
    const double u = 0x1p-53;
    double per = 2.0 * u;  // the factor's own rounding and the product's
    if (tri) {
        const double pm = 1.0 - p - pd;
        if (pm > 0.0) per = u * (2.0 + (1.0 - p) / pm);
    }
    // + 4 u: the powers p^a, (1-p)^(P-a) are library pow calls
    return steps * per + 10.0 * u;
}

// Relative part of the error bound of an exact result (see the reduction
// kernel): the prefix and suffix weights, the multiplier c_z, the clamped
// subtraction, every FP32 and FP64 sum on the way to the value, the
// discount.  Counts are of roundings a term passes through, each at most
// the unit roundoff of its precision relative to a sum of nonnegative terms.
static double rel_error_bound(const OptDev &d, int mode, bool tri, double rT)
{
    const double u = 0x1p-53, f = 0x1p-24;
    const double eW = weight_rel_err(d.P, tri, d.p, d.pd) + weight_rel_err(d.k, tri, d.p, d.pd);
    const double ec = d.eps_pre + 4.0 * u;  // c = W * cf * 2^e, cf from Pz
    // reduction: strided partial sums, wave tree, waves; the discount
    const double red = (double)((d.nitems + 255) / 256 + 11) + 3.0 + std::fabs(rT);
    const double sep = (double)(d.chunk / 1024 + 24);  // sums of W U over a chunk
    double acc;
    if (mode == 0) {
        // subtraction, FMA chain over the chunk's prefixes, lane's kJ suffixes
        acc = u * (1.0 + d.chunk + kJ + 2 + 6 + red + sep);
    } else if (mode == 3) {
        // subtraction, add chain over a group's prefixes in the chunk, the
        // omega-weighted fold of the lane's kJ group sums, the chain of up
        // to P + 1 group folds (W_a times the fold), the separable part
        acc = u * (1.0 + d.chunk + kJ + 1.0 + (d.P + 1.0) + kJ + 1 + 6 + red + sep);
    } else if (mode == 2) {
        // FP32: subtraction, a 16-leaf tree, the chain of a run's trees, the
        // Kahan fold of at most nrun runs per group and lane (2 f + 2 nrun
        // f^2); FP64: group flushes over the lane's suffixes and up to P + 1
        // groups, then as above
        const double nrun = (double)(d.chunk / (kBlock * kRunBlocks) + 1);
        acc = f * (1.0 + 4.0 + (kRunBlocks - 1) + 2.0 + 2.0 * nrun * f) +
              u * (3.0 + (d.P + 1.0) * kJ + kJ + 1 + 6 + red + sep);
    } else {
        // FP32: subtraction, g's rounding, a chain of kKahanRun FMAs, the
        // Kahan fold; FP64 as above with per-suffix accumulators
        acc = f * (1.0 + 1.0 + kKahanRun + 3.0) +
              u * (3.0 + d.P + 1.0 + kJ + 2 + 6 + red + sep);
    }
    return eW + ec + acc;
}

constexpr int kMaxPrefixSteps = 26;  // <= the table kernel's unranking limit (32)
constexpr int64_t kMaxChunks = (int64_t)1 << 22;
constexpr int64_t kMaxSharedPartials = (int64_t)1 << 27;  // chunks x draws

static uint32_t up_threshold_of(double p)
{
    const double t = std::floor(std::ldexp(p, 32));
    if (t >= 4294967296.0) return 0xFFFFFFFFu;
    return t <= 0 ? 0u : (uint32_t)t;
}

static int plan_layout(const bt_option *opts, int n, int precision, const bt_tuning *tune,
                       PlanLayout &L, const PlanSpec *ps = nullptr)
{
    const bool f32 = precision == BT_FP32_KAHAN;
    const PlanSpec *ss = (ps && ps->shared) ? ps : nullptr;
    const bool tv = ps && ps->tv_u;
    const bool tri = ps && ps->tri;
    if (ss && n != 1) return BT_EINVAL;
    L.shared = ss != nullptr;
    L.tv = tv;
    L.mode = (tv || tri || ss) ? (f32 ? 1 : 0) : (f32 ? 2 : 3);
    L.tv_host.clear();
    if (tv) {
        L.tv_host.assign(ps->tv_u, ps->tv_u + opts[0].N);
        L.tv_host.insert(L.tv_host.end(), ps->tv_p, ps->tv_p + opts[0].N);
    }
    L.od.assign(n, OptDev{});
    L.toff.assign(n, TableOffsets{});
    L.tune.clear();
    L.goff.assign(n, {});
    L.table_off.assign(n, 0);
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        const bt_option &o = opts[i];
        bt_tuning t = resolve_tuning(o.N, precision, tune, ps && ps->one_tree_shape,
                                     ps ? ps->depth_table : nullptr);
        if (tri) {
            // 3^k suffixes per lane tile set: k = min(N, 10) unless asked
            t.k = (tune && tune->k) ? std::min(tune->k, o.N) : std::min(o.N, 10);
            if (t.k > kTriMaxSuffix || o.N - t.k > kTriMaxPrefix) return BT_ERANGE;
        }
        if ((tri || tv) && !(tune && tune->chunk)) {
            // Chunks of about npre / 128 prefixes give one option enough
            // rectangles to fill the GPU; the shape depends on the option
            // alone, so an option prices the same in a plan of several.
            const int64_t np = ipow(tri ? 3 : 2, o.N - t.k);
            t.chunk = (int32_t)std::min<int64_t>(kMaxChunk, std::max<int64_t>(64, np / 128));
        }
        if (ss) {
            // split fixed by the estimator: r prefix steps, N - r drawn ones
            t.k = o.N - ss->r;
            const int64_t np = (int64_t)1 << ss->r;
            const int64_t div = f32 ? 64 : 32;
            t.chunk = (tune && tune->chunk) ? tune->chunk
                                            : (int32_t)std::min<int64_t>(kMaxChunk, std::max<int64_t>(64, np / div));
        }
        OptDev &d = L.od[i];
        std::memset(&d, 0, sizeof(d));
        d.S = o.S; d.u = o.u; d.p = o.p; d.K = o.K;
        d.disc = std::exp(-o.r * o.T);
        d.N = o.N; d.k = t.k; d.P = o.N - t.k; d.payoff = o.payoff;
        d.sign = sign_of(o.payoff);
        // X and Y are centred before scaling so that the FP32 form rounds
        // small numbers: an Asian suffix sum is near k, every other operand
        // (price ratios, multipliers) near 1; the difference is unchanged.
        d.center = (o.payoff == ASIAN_CALL || o.payoff == ASIAN_PUT) ? (double)t.k : 1.0;
        const int e = scale_exponent(o, d.P, d.k, d.center);
        d.scale = std::ldexp(1.0, e);
        d.inv_scale = std::ldexp(1.0, -e);
        d.base = tri ? 3 : 2;
        d.pd = tri ? ps->pd : 0.0;
        d.npre = ipow(d.base, d.P);
        d.nsuf = ss ? ss->R : ipow(d.base, d.k);
        d.tiles = (int32_t)((d.nsuf + kTile - 1) / kTile);
        d.chunk = (int32_t)std::min<int64_t>(t.chunk, d.npre);
        d.nchunks = (int32_t)((d.npre + d.chunk - 1) / d.chunk);
        // With fewer tiles than waves, the waves of a workgroup split the
        // chunk's prefixes instead of idling: one partial per part.
        d.wsplit = d.tiles < kWaves ? kWaves / d.tiles : 1;
        d.nitems = (int64_t)d.tiles * d.nchunks * d.wsplit;
        d.groups = (d.tiles + kWaves - 1) / kWaves;
        d.nbitems = (int64_t)d.nchunks * d.groups;
        d.out_index = i;
        d.fp32 = f32 ? 1 : 0;
        d.xonly = L.mode == 2 ? 1 : 0;
        d.ucount = ((f32 && !tv && !tri) || L.mode == 3) ? 1 : 0;
        const int64_t sufjob = suffix_job_size(tv, tri, ss != nullptr, d.xonly != 0);
        d.nsufjobs = (int32_t)((d.nsuf + sufjob - 1) / sufjob);
        d.eps_pre = (d.P + 6) * 0x1p-53;
        d.eps_suf = (d.k + 6) * 0x1p-53;
        // Size limits, checked before anything is built: the prefix table
        // (2^P records) and the number of chunks (one table workgroup each).
        if (d.P > kMaxPrefixSteps || d.nchunks > kMaxChunks) return BT_ERANGE;
        if ((tv || tri) && f32) {
            // FP32 keeps W_z in g_z: scale so that the largest weight is
            // near 1; refuse nonzero weights spread beyond 2^100 (FP32 range).
            double lo = 0.0, hi = 0.0;  // log2 of the smallest / largest W_z
            for (int t = 0; t < d.P; ++t) {
                double qmin, qmax;
                if (tv) {
                    const double q = ps->tv_p[t];
                    qmin = std::min(q, 1.0 - q);
                    qmax = std::max(q, 1.0 - q);
                } else {
                    const double pm = 1.0 - o.p - ps->pd;
                    qmin = std::min(o.p, ps->pd);
                    if (pm > 0.0) qmin = std::min(qmin, pm);
                    qmax = std::max(std::max(o.p, ps->pd), pm);
                }
                lo += std::log2(qmin);
                hi += std::log2(qmax);
            }
            if (hi - lo > 100.0) return BT_ERANGE;
            d.wexp = -(int32_t)std::floor(hi);
        }
        if (ss) {
            if ((int64_t)d.nchunks * d.wsplit * d.nsuf > kMaxSharedPartials) return BT_ERANGE;
            d.seed = ss->seed;
            d.stream_id = ss->stream_id;
            d.thr = up_threshold_of(o.p);
        }
        // table offsets, from the start of the plan's memory
        size_t q = total;
        auto put = [&](size_t bytes) { const size_t at = q; q += align256(bytes); return at; };
        TableOffsets &to = L.toff[i];
        to.X = put(d.npre * (d.xonly ? 4 : (f32 || d.ucount) ? 8 : 16));
        to.Y = put(d.nsuf * 8);
        to.Om = put(d.nsuf * 8);
        to.E = put(d.nsuf * 8);
        to.Y32 = f32 ? put(d.nsuf * 4) : 0;
        to.CU = put(d.nchunks * 8);
        to.Wg = put((d.P + 1) * 8);
        to.G = put((d.P + 2) * 8 + (d.P + 1) * 8);  // goff, then the group centres Cg
        to.PS = ss ? put((size_t)d.nchunks * d.wsplit * d.nsuf * 8) : 0;
        to.TV = tv ? put((size_t)2 * d.N * 8) : 0;
        to.BP = ss ? 0 : put((size_t)d.nchunks * 4 * 8);
        to.BS = ss ? 0 : put((size_t)d.nsufjobs * 4 * 8);
        // FP32 binomial bound: one suffix histogram per suffix job
        to.HS = (!ss && d.xonly) ? put((size_t)d.nsufjobs * 3 * kHistBins * 8) : 0;
        to.end = q;
        L.table_off[i] = total;
        total = q;
        // group offsets goff[0..P+1], then (bit for bit) the centres Cg[0..P]
        std::vector<int64_t> g(2 * d.P + 3, 0);
        int64_t c = 1;  // C(P, a)
        for (int a = 0; a <= d.P; ++a) {
            // time-varying moves, trinomial trees: one group (natural order)
            g[a + 1] = (tv || tri) ? d.npre : g[a] + c;
            c = c * (d.P - a) / (a + 1);
            const double cg = d.xonly ? group_centre(o, d, a) : 0.0;
            std::memcpy(&g[d.P + 2 + a], &cg, 8);
        }
        L.goff[i] = std::move(g);
        d.eY = d.xonly ? suffix_y_error(d, o.u) : 0.0;
        if (d.xonly) suffix_v_range(o, d, &d.vlo, &d.hw);
        L.tune.push_back(t);
        d.eps_rel = rel_error_bound(d, L.mode, tri, o.r * o.T);
    }
    // LPT order: largest workgroup item first, then most items.
    L.order.resize(n);
    for (int i = 0; i < n; ++i) L.order[i] = i;
    auto work = [&](const OptDev &d) {
        return std::min<int64_t>((int64_t)kTile * kWaves, d.nsuf) * d.chunk;
    };
    std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) {
        const int64_t wa = work(L.od[a]), wb = work(L.od[b]);
        if (wa != wb) return wa > wb;
        return L.od[a].nbitems > L.od[b].nbitems;
    });
    std::vector<int> pos(n);
    int64_t nitems = 0, nbitems = 0, nchunks = 0;
    for (int j = 0; j < n; ++j) {
        const int idx = L.order[j];
        pos[idx] = j;
        L.od[idx].item_begin = nitems;
        L.od[idx].bitem_begin = nbitems;
        L.od[idx].xa = xcd_blocking(L.od[idx], L.mode, nbitems);
        L.od[idx].chunk_begin = nchunks;
        nitems += L.od[idx].nitems;
        nbitems += L.od[idx].nbitems;
        nchunks += L.od[idx].nchunks;
    }
    L.nbitems = nbitems;
    L.nitems = nitems;
    L.nchunks = nchunks;
    L.jobs.clear();
    for (int i = 0; i < n; ++i) {
        const OptDev &d = L.od[i];
        for (int64_t c = 0; c < d.nchunks; ++c) {
            const int64_t first = c * d.chunk;
            L.jobs.push_back({pos[i], TAB_PREFIX, first, std::min<int64_t>(d.chunk, d.npre - first), c});
        }
        // Suffix blocks (suffix_job_size); a suffix job's `chunk` is its
        // index among the option's suffix jobs (its error-bound slot).
        const int64_t sufjob = suffix_job_size(L.tv, d.base == 3, L.shared, d.xonly != 0);
        for (int64_t s = 0; s < d.nsuf; s += sufjob)
            L.jobs.push_back({pos[i], TAB_SUFFIX, s, std::min<int64_t>(sufjob, d.nsuf - s),
                              s / sufjob});
        L.jobs.push_back({pos[i], TAB_WEIGHTS, 0, 0, 0});
    }
    L.off_partial = align256(total);
    L.off_counter = L.off_partial + align256((size_t)nitems * 8);
    L.off_values = L.off_counter + 256;
    L.off_od = L.off_values + align256((size_t)n * 2 * 8);  // values, then bounds
    L.off_jobs = L.off_od + align256(sizeof(OptDev) * n);
    L.total = L.off_jobs + align256(sizeof(TableJob) * L.jobs.size());
    return BT_OK;
}

// Host-side check, before anything is launched, that every array a kernel
// indexes lies inside the plan's memory with the extent the kernels assume
// (prefix records 2^P, suffix arrays 2^k, chunk sums, P+1 weights, P+2 group
// offsets, one partial per work item) and that no two overlap.
static int verify_layout(const PlanLayout &L, const char *mem, size_t bytes, int precision)
{
    const bool f32 = precision == BT_FP32_KAHAN;
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    auto inside = [&](const void *p, size_t n) {
        if (!p) return false;
        const uintptr_t a = reinterpret_cast<uintptr_t>(p), lo = reinterpret_cast<uintptr_t>(mem);
        if (a < lo || a + n > lo + bytes) return false;
        spans.emplace_back(a, a + n);
        return true;
    };
    int64_t items = 0, bitems = 0;
    for (const OptDev &d : L.od) {
        if (d.P < 0 || d.k < 1 || d.P + d.k != d.N || (d.base != 2 && d.base != 3) ||
            d.npre != ipow(d.base, d.P) ||
            (!L.shared && d.nsuf != ipow(d.base, d.k)) || d.nsuf < 1 || d.chunk < 1 || d.tiles < 1 ||
            (int64_t)d.nchunks * d.chunk < d.npre || (int64_t)(d.nchunks - 1) * d.chunk >= d.npre ||
            d.wsplit != (d.tiles < kWaves ? kWaves / d.tiles : 1) ||
            d.nitems != (int64_t)d.tiles * d.nchunks * d.wsplit || (int64_t)d.tiles * kTile < d.nsuf)
            return BT_EINVAL;
        bool ok = d.xonly == (L.mode == 2 ? 1 : 0) &&
                  d.ucount == (((f32 && !L.tv && d.base == 2) || L.mode == 3) ? 1 : 0) &&
                  d.nsufjobs == (d.nsuf + suffix_job_size(L.tv, d.base == 3, L.shared, d.xonly != 0) - 1) /
                                    suffix_job_size(L.tv, d.base == 3, L.shared, d.xonly != 0);
        if (f32) ok = ok && inside(d.XG, d.npre * (d.xonly ? 4 : 8)) && inside(d.Y32, d.nsuf * 4);
        else ok = ok && inside(d.XC, d.npre * (d.ucount ? 8 : 16));
        if (L.shared) ok = ok && !d.bnd_pre && !d.bnd_suf;
        else ok = ok && inside(d.bnd_pre, (size_t)d.nchunks * 32) &&
                  inside(d.bnd_suf, (size_t)d.nsufjobs * 32);
        ok = ok && inside(d.Y, d.nsuf * 8) && inside(d.Om, d.nsuf * 8) && inside(d.E, d.nsuf * 8) &&
             inside(d.chunkU, d.nchunks * 8) && inside(d.Wg, (d.P + 1) * 8) &&
             inside(d.goff, (d.P + 2) * 8 + (d.P + 1) * 8) &&
             d.Cg == reinterpret_cast<const double *>(d.goff + d.P + 2);
        if (d.xonly && !L.shared) ok = ok && inside(d.hist, (size_t)d.nsufjobs * 3 * kHistBins * 8);
        else ok = ok && !d.hist;
        if (L.shared) ok = ok && inside(d.persuf, (size_t)d.nchunks * d.wsplit * d.nsuf * 8);
        else ok = ok && !d.persuf;
        if (L.tv) ok = ok && inside(d.tv, (size_t)2 * d.N * 8);
        else ok = ok && !d.tv;
        if (!ok) return BT_EINVAL;
        if (d.item_begin < 0 || d.item_begin + d.nitems > L.nitems) return BT_EINVAL;
        if (d.chunk > kMaxChunk || d.groups < 1 || (int64_t)d.groups * kWaves < d.tiles ||
            d.nbitems != (int64_t)d.nchunks * d.groups || d.bitem_begin < 0 ||
            d.bitem_begin + d.nbitems > L.nbitems)
            return BT_EINVAL;
        items += d.nitems;
        bitems += d.nbitems;
    }
    if (items != L.nitems || bitems != L.nbitems) return BT_EINVAL;
    if (!inside(mem + L.off_partial, (size_t)L.nitems * 8) || !inside(mem + L.off_counter, 8) ||
        !inside(mem + L.off_values, L.od.size() * 2 * 8) ||
        !inside(mem + L.off_od, sizeof(OptDev) * L.od.size()) ||
        !inside(mem + L.off_jobs, sizeof(TableJob) * L.jobs.size()))
        return BT_EINVAL;
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return BT_EINVAL;
    for (const TableJob &j : L.jobs) {
        if (j.opt < 0 || j.opt >= (int)L.od.size()) return BT_EINVAL;
        const OptDev &d = L.od[L.order[j.opt]];
        if (j.kind == TAB_PREFIX && (j.first < 0 || j.count < 1 || j.first + j.count > d.npre ||
                                     j.chunk < 0 || j.chunk >= d.nchunks))
            return BT_EINVAL;
        if (j.kind == TAB_SUFFIX && (j.first < 0 || j.count < 1 || j.first + j.count > d.nsuf ||
                                     j.chunk < 0 || j.chunk >= d.nsufjobs))
            return BT_EINVAL;
    }
    return BT_OK;
}

static void assign_pointers(PlanLayout &L, char *base, int precision)
{
    for (size_t i = 0; i < L.od.size(); ++i) {
        OptDev &d = L.od[i];
        const TableOffsets &to = L.toff[i];
        if (precision == BT_FP32_KAHAN) {
            d.XG = reinterpret_cast<float *>(base + to.X);
            d.Y32 = reinterpret_cast<float *>(base + to.Y32);
        } else {
            d.XC = reinterpret_cast<double *>(base + to.X);
        }
        d.Y = reinterpret_cast<double *>(base + to.Y);
        d.Om = reinterpret_cast<double *>(base + to.Om);
        d.E = reinterpret_cast<double *>(base + to.E);
        d.chunkU = reinterpret_cast<double *>(base + to.CU);
        d.Wg = reinterpret_cast<double *>(base + to.Wg);
        d.goff = reinterpret_cast<int64_t *>(base + to.G);
        d.Cg = reinterpret_cast<double *>(base + to.G + (d.P + 2) * 8);
        d.hist = to.HS ? reinterpret_cast<uint64_t *>(base + to.HS) : nullptr;
        d.persuf = L.shared ? reinterpret_cast<double *>(base + to.PS) : nullptr;
        d.tv = L.tv ? reinterpret_cast<const double *>(base + to.TV) : nullptr;
        d.bnd_pre = L.shared ? nullptr : reinterpret_cast<double *>(base + to.BP);
        d.bnd_suf = L.shared ? nullptr : reinterpret_cast<double *>(base + to.BS);
    }
}

static int validate_plan_args(const bt_option *opts, int32_t n, int32_t precision,
                              const bt_tuning *tune, const PlanSpec *ps = nullptr)
{
    if (!opts || n < 1 || (precision != BT_FP64 && precision != BT_FP32_KAHAN)) return BT_EINVAL;
    const PlanSpec *ss = (ps && ps->shared) ? ps : nullptr;
    if (ss && n != 1) return BT_EINVAL;
    if (ss && (ss->R < 1 || ss->r < 0 || ss->r >= opts[0].N)) return BT_EINVAL;
    if (ps && (ps->tv_u != nullptr) != (ps->tv_p != nullptr)) return BT_EINVAL;
    if (ps && ps->tri) {
        if (ps->shared || ps->tv_u || !(ps->pd > 0.0)) return BT_EINVAL;
        for (int i = 0; i < n; ++i) {
            if (!(opts[i].p + ps->pd <= 1.0)) return BT_EINVAL;
            if (opts[i].N > kTriMaxN) return BT_ERANGE;
        }
    }
    if (ps && ps->tv_u) {
        // one step sequence for every option: all have its length
        for (int i = 1; i < n; ++i)
            if (opts[i].N != opts[0].N) return BT_EINVAL;
        if (opts[0].N < 1 || opts[0].N > kMcMaxN) return BT_ERANGE;
        for (int t = 0; t < opts[0].N; ++t)
            if (!(ps->tv_u[t] > 1.0) || !std::isfinite(ps->tv_u[t]) || !(ps->tv_p[t] > 0.0) ||
                !(ps->tv_p[t] < 1.0))
                return BT_EINVAL;
    }
    for (int i = 0; i < n; ++i) {
        const int rc = check_option(&opts[i], ss ? kMcMaxN : kExactMaxN);
        if (rc) return rc;
    }
    return check_tuning(tune);
}

int plan_bytes(const bt_option *opts, int32_t n, int32_t precision, const bt_tuning *tune,
               size_t *bytes, const PlanSpec *ss)
{
    int rc = validate_plan_args(opts, n, precision, tune, ss);
    if (rc) return rc;
    PlanLayout L;
    rc = plan_layout(opts, n, precision, tune, L, ss);
    if (rc) return rc;
    // The same layout checks run here, on the host, against a notional base
    // address, so that a bad layout is refused before any device exists.
    char *fake = reinterpret_cast<char *>((uintptr_t)1 << 40);
    assign_pointers(L, fake, precision);
    rc = verify_layout(L, fake, L.total, precision);
    if (rc) return rc;
    *bytes = L.total;
    return BT_OK;
}

// Build a plan in `mem` (device, >= plan_bytes); uploads are enqueued on s.
int plan_create_in(const bt_option *opts, int32_t n, int32_t precision, const bt_tuning *tune,
                   void *mem, size_t bytes, bool owns, hipStream_t s, bt_plan **out,
                   const PlanSpec *ss)
{
    *out = nullptr;
    int rc = validate_plan_args(opts, n, precision, tune, ss);
    if (rc) return rc;
    DeviceInfo *dev = nullptr;
    rc = ensure_device(&dev);
    if (rc) return rc;
    bt_plan *pl = new (std::nothrow) bt_plan();
    if (!pl) return BT_ENOMEM;
    PlanLayout L;
    rc = plan_layout(opts, n, precision, tune, L, ss);
    if (rc) { delete pl; return rc; }
    if (bytes < L.total) { delete pl; return BT_ENOMEM; }
    pl->device = dev->device;
    pl->precision = precision;
    pl->n = n;
    pl->mem = static_cast<char *>(mem);
    pl->owns_memory = owns;
    char *base = pl->mem;
    assign_pointers(L, base, precision);
    rc = verify_layout(L, base, bytes, precision);
    if (rc) {
        delete pl;
        return rc;
    }
    pl->d_partial = reinterpret_cast<double *>(base + L.off_partial);
    pl->d_counter = reinterpret_cast<unsigned long long *>(base + L.off_counter);
    pl->d_values = reinterpret_cast<double *>(base + L.off_values);
    pl->d_od = reinterpret_cast<OptDev *>(base + L.off_od);
    pl->d_jobs = reinterpret_cast<TableJob *>(base + L.off_jobs);
    pl->nitems = L.nitems;
    pl->nbitems = L.nbitems;
    pl->mode = L.mode;
    pl->bounds = !L.shared;
    pl->bound_chunks = (L.mode == 2 && !L.shared) ? L.nchunks : 0;
    pl->od.resize(n);
    for (int j = 0; j < n; ++j) pl->od[j] = L.od[L.order[j]];
    pl->jobs = L.jobs;
    pl->table_entries = job_entries(L.jobs);
    pl->tune = L.tune;
    pl->status.assign(n, BT_OK);
    // Uploads from host copies that live as long as the plan.
    pl->host_goff = std::move(L.goff);
    bool ok = hipMemcpyAsync(pl->d_od, pl->od.data(), sizeof(OptDev) * n, hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(pl->d_jobs, pl->jobs.data(), sizeof(TableJob) * pl->jobs.size(),
                             hipMemcpyHostToDevice, s) == hipSuccess;
    for (int i = 0; i < n && ok; ++i)
        ok = hipMemcpyAsync(L.od[i].goff, pl->host_goff[i].data(), pl->host_goff[i].size() * 8,
                            hipMemcpyHostToDevice, s) == hipSuccess;
    pl->host_tv = std::move(L.tv_host);
    for (int i = 0; ok && L.tv && i < n; ++i)  // each option's copy of the steps
        ok = hipMemcpyAsync(const_cast<double *>(L.od[i].tv), pl->host_tv.data(),
                            pl->host_tv.size() * 8, hipMemcpyHostToDevice, s) == hipSuccess;
    if (!ok) {
        pl->owns_memory = false;
        bt_plan_destroy(pl);
        return BT_EDEVICE;
    }
    const bool f32 = precision == BT_FP32_KAHAN;
    pl->waves = kWaves;
    (void)f32;
    // Default: one workgroup per rectangle; a smaller grid makes each
    // workgroup loop over rectangles g, g + grid, ...
    const int64_t max_grid = (int64_t)1 << 30;
    int64_t grid = (tune && tune->grid) ? tune->grid : std::min<int64_t>(pl->nbitems, max_grid);
    if (grid > pl->nbitems) grid = std::max<int64_t>(1, pl->nbitems);
    pl->grid = (int)grid;
    pl->used = pl->tune[0];
    pl->used.grid = (int32_t)grid;
    pl->used.waves = kWaves;
    *out = pl;
    return BT_OK;
}

}  // namespace bt

namespace bt {
static int plan_create_owned(const bt_option *opts, int32_t n, int32_t precision,
                             const bt_tuning *tune, bt_plan **out, const PlanSpec *ps);
}  // namespace bt

extern "C" int bt_plan_create(const bt_option *opts, int32_t n, int32_t precision,
                              const bt_tuning *tune, bt_plan **out)
{
    if (!out) return BT_EINVAL;
    return plan_create_owned(opts, n, precision, tune, out, nullptr);
}

extern "C" int bt_plan_tables(bt_plan *plan, void *stream)
{
    if (!plan) return BT_EINVAL;
    return hip_err(launch_tables(plan->d_od, plan->d_jobs, (int)plan->jobs.size(),
                                 plan->table_entries, (hipStream_t)stream));
}

extern "C" int bt_plan_enumerate(bt_plan *plan, void *stream)
{
    if (!plan) return BT_EINVAL;
    return hip_err(launch_enumerate(plan->d_od, plan->n, plan->nbitems, plan->d_partial,
                                    plan->mode, plan->grid, plan->bound_chunks,
                                    (hipStream_t)stream));
}

extern "C" int bt_plan_reduce(bt_plan *plan, void *stream)
{
    if (!plan) return BT_EINVAL;
    return hip_err(launch_reduce(plan->d_od, plan->n, plan->d_partial, plan->d_values,
                                 (hipStream_t)stream));
}

extern "C" int bt_plan_results(bt_plan *plan, bt_result *outs, void *stream)
{
    if (!plan || !outs) return BT_EINVAL;
    std::vector<double> v(2 * (size_t)plan->n);
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(v.data(), plan->d_values, sizeof(double) * 2 * plan->n,
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return BT_EDEVICE;
    for (int j = 0; j < plan->n; ++j) {
        const OptDev &d = plan->od[j];
        bt_result &r = outs[d.out_index];
        std::memset(&r, 0, sizeof(r));
        r.value = v[d.out_index];
        r.err_bound = plan->bounds ? v[plan->n + d.out_index] : NAN;
        r.paths = (uint64_t)d.npre * (uint64_t)d.nsuf;
        r.split = d.k;
        r.status = plan->status[d.out_index];
    }
    return BT_OK;
}

extern "C" int bt_plan_device_values(bt_plan *plan, double **d_values)
{
    if (!plan || !d_values) return BT_EINVAL;
    *d_values = plan->d_values;
    return BT_OK;
}

extern "C" int bt_plan_info(const bt_plan *plan, uint64_t *items, bt_tuning *used)
{
    if (!plan) return BT_EINVAL;
    if (items) *items = (uint64_t)plan->nitems;
    if (used) *used = plan->used;
    return BT_OK;
}

extern "C" int bt_plan_capture(bt_plan *plan, void *stream)
{
    if (!plan || !stream) return BT_EINVAL;  // the legacy stream cannot be captured
    hipStream_t s = (hipStream_t)stream;
    if (plan->gexec) { (void)hipGraphExecDestroy(plan->gexec); plan->gexec = nullptr; }
    if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return BT_EDEVICE;
    int rc = bt_plan_tables(plan, s);
    if (!rc) rc = bt_plan_enumerate(plan, s);
    if (!rc) rc = bt_plan_reduce(plan, s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : BT_EDEVICE;
    }
    if (hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        plan->gexec = nullptr;
        return BT_EDEVICE;
    }
    plan->graph = g;
    return BT_OK;
}

extern "C" int bt_plan_launch_graph(bt_plan *plan, void *stream)
{
    if (!plan || !plan->gexec) return BT_EINVAL;
    return hip_err(hipGraphLaunch(plan->gexec, (hipStream_t)stream));
}

extern "C" int bt_plan_debug_tables(bt_plan *plan, int32_t i, uint64_t *prefix_z,
                                    int32_t *prefix_a, int32_t *suffix_b, void *stream)
{
    if (!plan || i < 0 || i >= plan->n || !prefix_z || !prefix_a || !suffix_b) return BT_EINVAL;
    int j = 0;
    while (j < plan->n && plan->od[j].out_index != i) ++j;
    OptDev d = plan->od[j];
    hipStream_t s = (hipStream_t)stream;
    char *buf = nullptr;
    const size_t bz = align256(d.npre * 8), ba = align256(d.npre * 4), bb = align256(d.nsuf * 4);
    if (hipMalloc(&buf, bz + ba + bb) != hipSuccess) return BT_ENOMEM;
    d.dbg_z = reinterpret_cast<uint64_t *>(buf);
    d.dbg_a = reinterpret_cast<int32_t *>(buf + bz);
    d.dbg_b = reinterpret_cast<int32_t *>(buf + bz + ba);
    int rc = BT_OK;
    OptDev *d_one = nullptr;
    TableJob *d_j = nullptr;
    std::vector<TableJob> jobs;
    for (const TableJob &jb : plan->jobs)
        if (jb.opt == j) { TableJob t = jb; t.opt = 0; jobs.push_back(t); }
    if (hipMalloc(&d_one, sizeof(OptDev)) != hipSuccess ||
        hipMalloc(&d_j, sizeof(TableJob) * jobs.size()) != hipSuccess) {
        rc = BT_ENOMEM;
    } else if (hipMemcpy(d_one, &d, sizeof(OptDev), hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(d_j, jobs.data(), sizeof(TableJob) * jobs.size(), hipMemcpyHostToDevice) != hipSuccess ||
               launch_tables(d_one, d_j, (int)jobs.size(), job_entries(jobs), s) != hipSuccess ||
               hipStreamSynchronize(s) != hipSuccess ||
               hipMemcpy(prefix_z, d.dbg_z, d.npre * 8, hipMemcpyDeviceToHost) != hipSuccess ||
               hipMemcpy(prefix_a, d.dbg_a, d.npre * 4, hipMemcpyDeviceToHost) != hipSuccess ||
               hipMemcpy(suffix_b, d.dbg_b, d.nsuf * 4, hipMemcpyDeviceToHost) != hipSuccess) {
        rc = BT_EDEVICE;
    }
    if (d_one) (void)hipFree(d_one);
    if (d_j) (void)hipFree(d_j);
    (void)hipFree(buf);
    return rc;
}

// ------------------------------------------------------------------ one-shot

namespace bt {

int plan_price_in(const bt_option *opts, int32_t n, int32_t precision, const bt_tuning *tune,
                  bt_result *outs, void *mem, size_t bytes, hipStream_t s, const PlanSpec *ps)
{
    bt_plan *pl = nullptr;
    int rc = plan_create_in(opts, n, precision, tune, mem, bytes, false, s, &pl, ps);
    if (!rc) rc = bt_plan_tables(pl, s);
    if (!rc) rc = bt_plan_enumerate(pl, s);
    if (!rc) rc = bt_plan_reduce(pl, s);
    if (!rc) rc = bt_plan_results(pl, outs, s);  // synchronizes s
    else (void)hipStreamSynchronize(s);          // nothing may still use mem
    if (pl) bt_plan_destroy(pl);                 // host state only
    return rc;
}

// The one-shot calls: a plan in a buffer of the library's per-device cache.
static int price_pooled(const bt_option *opts, int32_t n, int32_t precision,
                        const bt_tuning *tune, bt_result *outs, hipStream_t s,
                        const PlanSpec *ps = nullptr)
{
    size_t bytes = 0;
    int rc = plan_bytes(opts, n, precision, tune, &bytes, ps);
    if (rc) return rc;
    rc = ensure_device(nullptr);
    if (rc) return rc;
    void *mem = nullptr;
    size_t cap = 0;
    rc = pool_acquire(bytes, &mem, &cap);
    if (rc) return rc;
    rc = plan_price_in(opts, n, precision, tune, outs, mem, cap, s, ps);
    pool_release(mem);
    return rc;
}

// Time-varying moves: every option takes the largest step factor as its u
// (what the layout's scale needs) and p_1 as its p (checked, then unused);
// the steps themselves travel in the PlanSpec.
static int tv_prepare(const bt_option *opts, int32_t n, const double *u_t, const double *p_t,
                      std::vector<bt_option> &o, PlanSpec &ps)
{
    if (!opts || n < 1 || !u_t || !p_t || opts[0].N < 1) return BT_EINVAL;
    if (opts[0].N > kExactMaxN) return BT_ERANGE;
    double umax = 0.0;
    for (int t = 0; t < opts[0].N; ++t) {
        if (!(u_t[t] > 1.0) || !std::isfinite(u_t[t]) || !(p_t[t] > 0.0) || !(p_t[t] < 1.0))
            return BT_EINVAL;
        umax = std::max(umax, u_t[t]);
    }
    o.assign(opts, opts + n);
    for (bt_option &x : o) {
        if (x.N != opts[0].N) return BT_EINVAL;
        x.u = umax;
        x.p = p_t[0];
    }
    ps.tv_u = u_t;
    ps.tv_p = p_t;
    return BT_OK;
}

// A plan that owns a fresh allocation (bt_plan_create and its forms).
static int plan_create_owned(const bt_option *opts, int32_t n, int32_t precision,
                             const bt_tuning *tune, bt_plan **out, const PlanSpec *ps)
{
    *out = nullptr;
    size_t bytes = 0;
    int rc = plan_bytes(opts, n, precision, tune, &bytes, ps);
    if (rc) return rc;
    rc = ensure_device(nullptr);
    if (rc) return rc;
    void *mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return BT_ENOMEM;
    rc = plan_create_in(opts, n, precision, tune, mem, bytes, true, nullptr, out, ps);
    if (rc) {
        (void)hipStreamSynchronize(nullptr);
        (void)hipFree(mem);
        return rc;
    }
    if (hipStreamSynchronize(nullptr) != hipSuccess) {
        bt_plan_destroy(*out);
        *out = nullptr;
        return BT_EDEVICE;
    }
    return BT_OK;
}

}  // namespace bt

extern "C" int bt_plan_bytes(const bt_option *opts, int32_t n, int32_t precision,
                             const bt_tuning *tune, size_t *bytes)
{
    if (!bytes) return BT_EINVAL;
    return plan_bytes(opts, n, precision, tune, bytes);
}

extern "C" int bt_price_batch(const bt_option *opts, int32_t n, int32_t precision,
                              const bt_tuning *tune, bt_result *outs, void *stream)
{
    if (!opts || !outs || n < 1) return BT_EINVAL;
    return price_pooled(opts, n, precision, tune, outs, (hipStream_t)stream);
}

extern "C" int bt_price_exact(const bt_option *opt, int32_t precision, const bt_tuning *tune,
                              bt_result *out, void *stream)
{
    if (!opt || !out) return BT_EINVAL;
    return bt_price_batch(opt, 1, precision, tune, out, stream);
}

extern "C" int bt_price_batch_ws(const bt_option *opts, int32_t n, int32_t precision,
                                 const bt_tuning *tune, bt_result *outs, void *d_workspace,
                                 size_t ws_bytes, void *stream)
{
    if (!opts || !outs || n < 1 || !d_workspace || ((uintptr_t)d_workspace & 255)) return BT_EINVAL;
    size_t bytes = 0;
    int rc = plan_bytes(opts, n, precision, tune, &bytes);
    if (rc) return rc;
    if (bytes > ws_bytes) return BT_ENOMEM;
    rc = ensure_device(nullptr);
    if (rc) return rc;
    return plan_price_in(opts, n, precision, tune, outs, d_workspace, ws_bytes,
                         (hipStream_t)stream);
}

extern "C" int bt_price_exact_ws(const bt_option *opt, int32_t precision, const bt_tuning *tune,
                                 bt_result *out, void *d_workspace, size_t ws_bytes,
                                 void *stream)
{
    if (!opt || !out) return BT_EINVAL;
    return bt_price_batch_ws(opt, 1, precision, tune, out, d_workspace, ws_bytes, stream);
}

extern "C" int bt_plan_create_tv(const bt_option *opts, int32_t n, const double *u_t,
                                 const double *p_t, int32_t precision, const bt_tuning *tune,
                                 bt_plan **out)
{
    if (!out) return BT_EINVAL;
    *out = nullptr;
    std::vector<bt_option> o;
    PlanSpec ps;
    const int rc = tv_prepare(opts, n, u_t, p_t, o, ps);
    if (rc) return rc;
    return plan_create_owned(o.data(), n, precision, tune, out, &ps);
}

extern "C" int bt_price_exact_tv(const bt_option *opt, const double *u_t, const double *p_t,
                                 int32_t precision, const bt_tuning *tune, bt_result *out,
                                 void *stream)
{
    if (!out) return BT_EINVAL;
    std::vector<bt_option> o;
    PlanSpec ps;
    const int rc = tv_prepare(opt, 1, u_t, p_t, o, ps);
    if (rc) return rc;
    return price_pooled(o.data(), 1, precision, tune, out, (hipStream_t)stream, &ps);
}

extern "C" int bt_plan_create_trinomial(const bt_option *opts, int32_t n, double p_down,
                                        int32_t precision, const bt_tuning *tune, bt_plan **out)
{
    if (!out) return BT_EINVAL;
    *out = nullptr;
    if (!opts || n < 1) return BT_EINVAL;
    PlanSpec ps;
    ps.tri = true;
    ps.pd = p_down;
    return plan_create_owned(opts, n, precision, tune, out, &ps);
}

extern "C" int bt_price_exact_trinomial(const bt_option *opt, double p_down, int32_t precision,
                                        const bt_tuning *tune, bt_result *out, void *stream)
{
    if (!out || !opt) return BT_EINVAL;
    PlanSpec ps;
    ps.tri = true;
    ps.pd = p_down;
    return price_pooled(opt, 1, precision, tune, out, (hipStream_t)stream, &ps);
}

// ------------------------------------------------------------------ autotune

namespace {

// A tuning rule for every depth: k = (N + 1)/2 + dk within [8, 16] (all N
// for N <= 10) and chunks of max(cmin, 2^P / div) prefixes, at most
// kMaxChunk.  The autotuner picks one rule for a set of depths by the
// throughput of a whole batch, because launch shapes that look best for one
// small tree alone (where launch latency dominates) are not the ones that
// fill the GPU when thousands of trees share a launch.
struct TuneRule {
    int dk;
    int64_t cmin;
    int64_t div;
};

bt_tuning rule_tuning(const TuneRule &R, int N)
{
    bt_tuning t{};
    t.k = (N <= 10) ? N : std::min(16, std::max(8, (N + 1) / 2 + R.dk));
    t.k = std::min(t.k, N);
    const int64_t npre = (int64_t)1 << (N - t.k);
    t.chunk = (int32_t)std::min<int64_t>(kMaxChunk, std::max<int64_t>(R.cmin, npre / R.div));
    t.waves = kWaves;
    return t;
}

void install_rule(const TuneRule &R, int precision, int n_lo, int n_hi)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int N = n_lo; N <= n_hi; ++N) g_tuned[precision ? 1 : 0][N] = rule_tuning(R, N);
}

// Time tables + enumeration of the whole set under each rule (passed to the
// candidate's plan alone, so pricing on other threads never sees a
// candidate); install the fastest, once.  BT_EDEVICE if no candidate ran.
int tune_on_batch(const bt_option *opts, int32_t n, int32_t precision, hipStream_t s, int n_lo,
                  int n_hi)
{
    const TuneRule rules[] = {
        {0, 1024, 32}, {-1, 1024, 32}, {1, 1024, 32}, {-2, 1024, 32}, {2, 1024, 32},
        {0, 512, 32},  {0, 2048, 16},  {0, 1024, 64}, {-1, 2048, 16}, {1, 512, 64}};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return BT_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return BT_EDEVICE;
    }
    float best = 1e30f;
    int best_i = -1;
    int rc = BT_OK, first_err = BT_OK;
    std::vector<bt_tuning> table(kExactMaxN + 1);
    for (int i = 0; i < (int)(sizeof(rules) / sizeof(rules[0])); ++i) {
        std::fill(table.begin(), table.end(), bt_tuning{});
        for (int N = n_lo; N <= n_hi; ++N) table[N] = rule_tuning(rules[i], N);
        PlanSpec ps;
        ps.depth_table = table.data();
        bt_plan *pl = nullptr;
        const int prc = plan_create_owned(opts, n, precision, nullptr, &pl, &ps);
        if (prc) {
            if (!first_err) first_err = prc;
            continue;
        }
        bool ok = !bt_plan_tables(pl, s) && !bt_plan_enumerate(pl, s);
        float ms = 1e30f;
        for (int rep = 0; ok && rep < 2; ++rep) {
            ok = hipEventRecord(e0, s) == hipSuccess && !bt_plan_tables(pl, s) &&
                 !bt_plan_enumerate(pl, s) && hipEventRecord(e1, s) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess;
            float t_ms = 0;
            if (ok && hipEventElapsedTime(&t_ms, e0, e1) == hipSuccess) ms = std::min(ms, t_ms);
        }
        if (hipStreamSynchronize(s) != hipSuccess) rc = BT_EDEVICE;
        bt_plan_destroy(pl);
        if (ok && ms < best) {
            best = ms;
            best_i = i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_i < 0) return first_err ? first_err : BT_EDEVICE;
    install_rule(rules[best_i], precision, n_lo, n_hi);
    return rc;
}

}  // namespace

extern "C" int bt_autotune(int32_t n_lo, int32_t n_hi, int32_t precision, void *stream)
{
    if (n_lo < 1 || n_hi > kExactMaxN || n_lo > n_hi ||
        (precision != BT_FP64 && precision != BT_FP32_KAHAN))
        return BT_EINVAL;
    int rc = ensure_device(nullptr);
    if (rc) return rc;
    // A synthetic batch over the depths: about 2^34 / (number of depths)
    // paths per depth (Asian calls of the N=20 market), at most 4096 trees
    // per depth.
    const int nd = n_hi - n_lo + 1;
    std::vector<bt_option> opts;
    for (int N = n_lo; N <= n_hi; ++N) {
        double u = 0, p = 0;
        bt_params(0.2, 0.05, 1.0, N, BT_SCHEME_CRR, &u, &p);
        const double per = std::ldexp(1.0, 34) / nd;
        const int64_t copies = std::min<int64_t>(4096, std::max<int64_t>(1, (int64_t)(per / std::ldexp(1.0, N))));
        for (int64_t c = 0; c < copies; ++c)
            opts.push_back(bt_option{100.0, u, p, 0.05, 1.0, 90.0 + (double)(c % 21), N, BT_ASIAN_CALL});
    }
    return tune_on_batch(opts.data(), (int32_t)opts.size(), precision, (hipStream_t)stream, n_lo,
                         n_hi);
}

extern "C" int bt_autotune_batch(const bt_option *opts, int32_t n, int32_t precision,
                                 void *stream)
{
    if (!opts || n < 1 || (precision != BT_FP64 && precision != BT_FP32_KAHAN)) return BT_EINVAL;
    int n_lo = kExactMaxN + 1, n_hi = 0;
    for (int i = 0; i < n; ++i) {
        const int rc = check_option(&opts[i], kExactMaxN);
        if (rc) return rc;
        n_lo = std::min(n_lo, (int)opts[i].N);
        n_hi = std::max(n_hi, (int)opts[i].N);
    }
    int rc = ensure_device(nullptr);
    if (rc) return rc;
    return tune_on_batch(opts, n, precision, (hipStream_t)stream, n_lo, n_hi);
}

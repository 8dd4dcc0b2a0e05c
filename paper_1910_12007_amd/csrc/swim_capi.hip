// swim_capi.hip -- C ABI of libswim (declared in include/swim.h): argument
// checking, workspace, batch layout and longest-first scheduling, kernel
// launches, and the host FP64 parts of ABC / PMC.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/swim.h"
#include "swim_internal.h"
#include "swim_math.h"
#include "swim_philox.h"

using namespace swim;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// A failed HIP call is reported through the return code; HIP's per-thread
// last-error state is cleared so later, unrelated HIP users do not see it.
#define HIPCHK(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            (void)hipGetLastError();                                                       \
            return fail(SWIM_EHIP, "%s: %s", #call, hipGetErrorString(e_));                \
        }                                                                                  \
    } while (0)

#define TRY(expr)                 \
    do {                          \
        int rc_ = (expr);         \
        if (rc_ != SWIM_OK) return rc_; \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

enum BufId {
    B_OFF, B_SWOFF, B_NPT, B_NSW, B_ORDER, B_LIST, B_BLKS, B_BLKF, B_ALPHA, B_EPS, B_SYSC, B_QUEUE,
    B_PARAMS, B_DATA, B_OBS, B_SPEED, B_STATUS, B_DIST, B_TOL, B_ACC, B_BIG,
    B_MLP_ACT, B_MLP_GRAD, B_MLP_BATCH, B_MLP_IDX, B_MLP_CNT,
    B_PS_THETA, B_PS_X, B_PS_KEEP, B_PS_IDX, B_PS_NK, B_PS_SUM, B_DS_T, B_TAB, B_DONE, B_W16, B_SIGMA, B_LOGL,
    B_SP_SW, B_SP_HEAD, B_SP_TAIL, B_SP_G, B_SP_SIG, B_WTAB,
    B_BT_PSYS, B_BT_PT, B_BT_TSYS, B_BT_TT, B_BT_POFF, B_BT_PART,
    B_NBUF
};

// surrogate network: 5 -> 256 x 4 -> 33
constexpr int MLP_L = 5;
constexpr int MLP_W[MLP_L + 1] = {5, 256, 256, 256, 256, 33};
int64_t mlp_offW(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += (int64_t)MLP_W[k] * MLP_W[k + 1] + MLP_W[k + 1];
    return o;
}
int64_t mlp_offb(int l) { return mlp_offW(l) + (int64_t)MLP_W[l] * MLP_W[l + 1]; }
constexpr int64_t MLP_NPARAM = 207393;

}  // namespace

// Workspace of swim_pair_velocity_noalloc: a fixed device array in place of
// the context's allocations.  Sections (256-byte aligned): system offsets,
// alpha, eps, the block list (system, first target) of the pair kernel, the
// per-system constants (in the working type and in FP64) and the FP32 kernel
// tables.  Every section is written by the call before its kernels read it,
// so nothing needs clearing between calls.
constexpr int64_t NOALLOC_MAX_SYS = 64;      // systems per call
constexpr int64_t NOALLOC_MAX_BLOCKS = 4160; // pair-kernel blocks (256 targets each) per call
constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t NA_OFF = 0;
constexpr size_t NA_ALPHA = na_align(NA_OFF + (NOALLOC_MAX_SYS + 1) * 8);
constexpr size_t NA_EPS = na_align(NA_ALPHA + NOALLOC_MAX_SYS * 8);
constexpr size_t NA_BLKS = na_align(NA_EPS + NOALLOC_MAX_SYS * 8);
constexpr size_t NA_BLKF = na_align(NA_BLKS + NOALLOC_MAX_BLOCKS * 8);
constexpr size_t NA_SYSC = na_align(NA_BLKF + NOALLOC_MAX_BLOCKS * 8);  // end of the staged host data
constexpr size_t NA_SYSC64 = na_align(NA_SYSC + NOALLOC_MAX_SYS * sizeof(SysConst<double>));
constexpr size_t NA_TAB = na_align(NA_SYSC64 + NOALLOC_MAX_SYS * sizeof(SysConst<double>));
constexpr size_t NA_BYTES = na_align(NA_TAB + NOALLOC_MAX_SYS * sizeof(TabSys));  // ~1.7 MB

static_assert(sizeof(SysConst<float>) <= sizeof(SysConst<double>), "FP32 constants share the FP64 slots");
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

// The array's device address on each device, taken once per device by
// swim_create (hipGetSymbolAddress with that device current).  Host code
// uses these addresses, never the array's name.
constexpr int NOALLOC_MAX_DEV = 64;
static void* g_scratch_dev[NOALLOC_MAX_DEV];
static std::mutex g_scratch_mu;

// a captured forward-run launch sequence, replayed while its layout and
// buffers are unchanged
struct FwdGraph {
    uint64_t key = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};
constexpr int N_GRAPHS = 4;

struct swim_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 0;
    int opt_wps = 0;      // waves per system in the persistent kernel (0: automatic)
    int opt_big_tpl = 0;  // targets per lane of the large-system kernel (0: automatic)
    int opt_graph = 1;    // 0: eager launches; 1: capture on a repeated layout; 2: capture always
    int opt_blob = 1;     // 1: the paper's blob (eq. eqnblob); 0: the kernel reading's blob
    int opt_early_stop = 1;  // abc_prescreened stops re-runs whose distance already exceeds tol
    int tuned_wps[2][9] = {};  // autotuned waves per system [dtype][tpl] (0: not tuned)
    FwdGraph graphs[N_GRAPHS];
    uint64_t graph_clock = 0, last_key = 0;
    int64_t graph_launches = 0, graph_captures = 0;
    DevBuf buf[B_NBUF];
    void* pinned = nullptr;
    size_t pinned_cap = 0, pin_off = 0;
    hipEvent_t up_ev = nullptr;
    hipEvent_t sw_ev = nullptr;        // orders work across a change of stream
    // auxiliary streams (default priority) and events that run the size
    // buckets of one forward call side by side, forked from and joined to
    // the call's stream (in a captured graph: parallel branches)
    static constexpr int N_AUX = 3;
    hipStream_t aux[N_AUX] = {};
    hipEvent_t fork_ev = nullptr, join_ev[N_AUX] = {};
    // SWIM_OPT_TIME_KERNEL: timing events around the persistent launches of
    // the last forward call (its last chunk), read by SWIM_OPT_KERNEL_US
    int opt_time = 0;
    hipEvent_t time_ev[2] = {};
    bool timed = false;
    hipStream_t last_stream = nullptr;  // stream of the previous call (null: none yet)
    bool broken = false;
    // the autotuner's probes of one launch bucket alone: the bucket each
    // natural size bucket launches in, taken from the whole batch
    bool forced_launch = false;
    int force_launch_tpl[9] = {};
};

namespace {

int ensure(swim_ctx* c, BufId id, size_t bytes)
{
    DevBuf& b = c->buf[id];
    if (bytes <= b.cap) return SWIM_OK;
    if (b.p) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t cap = std::max<size_t>(bytes + bytes / 4, 256);
    if (hipMalloc(&b.p, cap) != hipSuccess) return fail(SWIM_ENOMEM, "device allocation of %zu bytes failed", cap);
    b.cap = cap;
    return SWIM_OK;
}

// Host->device staging through one pinned buffer.  begin_uploads waits for
// the previous call's copies, then stage() appends and enqueues copies.
int begin_uploads(swim_ctx* c, size_t total)
{
    HIPCHK(hipEventSynchronize(c->up_ev));
    c->pin_off = 0;
    total += 64 * 32;
    if (total > c->pinned_cap) {
        if (c->pinned) HIPCHK(hipHostFree(c->pinned));
        c->pinned = nullptr;
        c->pinned_cap = 0;
        size_t cap = total + total / 2;
        if (hipHostMalloc(&c->pinned, cap, hipHostMallocDefault) != hipSuccess)
            return fail(SWIM_ENOMEM, "pinned allocation of %zu bytes failed", cap);
        c->pinned_cap = cap;
    }
    return SWIM_OK;
}

int stage(swim_ctx* c, const void* src, size_t bytes, BufId dst, hipStream_t st)
{
    TRY(ensure(c, dst, bytes));
    if (bytes == 0) return SWIM_OK;
    c->pin_off = (c->pin_off + 63) & ~(size_t)63;
    if (c->pin_off + bytes > c->pinned_cap) return fail(SWIM_EINVAL, "internal: staging overflow");
    char* p = (char*)c->pinned + c->pin_off;
    memcpy(p, src, bytes);
    HIPCHK(hipMemcpyAsync(c->buf[dst].p, p, bytes, hipMemcpyHostToDevice, st));
    c->pin_off += bytes;
    return SWIM_OK;
}

int end_uploads(swim_ctx* c, hipStream_t st)
{
    HIPCHK(hipEventRecord(c->up_ev, st));
    return SWIM_OK;
}

// The stream a call runs on (null: the context's).  The context's device
// buffers (offsets, constants, tables, staging targets) are shared by every
// call, so when a call comes on another stream than the previous one, its
// stream first waits for everything enqueued so far on that previous stream:
// the new call's copies and kernels cannot overwrite buffers that kernels of
// the previous call are still reading.
hipStream_t pick(swim_ctx* c, void* s)
{
    hipStream_t st = s ? (hipStream_t)s : c->stream;
    if (c->last_stream && st != c->last_stream) {
        if (hipEventRecord(c->sw_ev, c->last_stream) != hipSuccess || hipStreamWaitEvent(st, c->sw_ev, 0) != hipSuccess) {
            // the previous stream is gone: its work was ordered by its destruction
            (void)hipGetLastError();
        }
    }
    c->last_stream = st;
    return st;
}

int check_ctx(swim_ctx* c)
{
    if (!c) return fail(SWIM_EINVAL, "null context");
    if (c->broken) return fail(SWIM_ESTATE, "context is unusable after an earlier HIP failure");
    HIPCHK(hipSetDevice(c->device));
    return SWIM_OK;
}

int check_dtype(int32_t d) { return (d == SWIM_F32 || d == SWIM_F64) ? SWIM_OK : fail(SWIM_EINVAL, "dtype must be SWIM_F32 or SWIM_F64"); }

// FNV-1a over the bytes that describe a launch layout
struct Fnv {
    uint64_t v = 1469598103934665603ull;
    void add_bytes(const void* p, size_t n)
    {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) {
            v ^= b[i];
            v *= 1099511628211ull;
        }
    }
    template <typename V> void add(const V& x) { add_bytes(&x, sizeof(x)); }
};

constexpr int TPL_CHOICES[] = {1, 2, 3, 4, 6, 8};
int choose_tpl(int pts)
{
    for (int t : TPL_CHOICES)
        if (pts <= 64 * t) return t;
    return -1;
}

// targets per lane of a forward system in the persistent kernel, or -1 for
// the large-system step: systems above 512 points, and FP32 systems whose
// pairs can lie beyond the FP32 kernel table after the first step (within
// the position bound pairs are at most 2829 apart, and the table holds
// v = 1 + (r / eps)^2 < 2^44, eps = eps_over_ds / (N - 1)): the persistent
// kernel reads the table without testing for such pairs, the large-system
// step evaluates them directly
int forward_tpl(int32_t dtype, int N, int pts, double eps_over_ds)
{
    if (dtype == SWIM_F32 && 2829.0 * (double)(N - 1) / eps_over_ds >= 4194304.0) return -1;
    return choose_tpl(pts);
}

// The targets per lane each size bucket launches with.  The buckets of one
// call (plus the large systems, big) run side by side on at most lanes
// streams.  With more parts than lanes, a lane would run two launches one
// after the other, the second waiting for the first one's tail (its longest
// run, one workgroup on part of a CU); instead, adjacent buckets merge until
// the parts fit, the smaller bucket's systems running in the larger one's
// kernel.  The pair merged is the one closest in size (the largest ratio of
// the two targets per lane; the larger sizes on a tie), whose smaller
// systems lose the least in the larger kernel.  present[t]: some system
// takes t targets per lane (choose_tpl); launch[t]: the targets per lane it
// runs with (0 where t is absent).
void merge_buckets(const bool (&present)[9], bool big, int lanes, int (&launch)[9])
{
    std::vector<int> ts;
    for (int t : TPL_CHOICES)
        if (present[t]) ts.push_back(t);
    while ((int)ts.size() + (big ? 1 : 0) > lanes && ts.size() > 1) {
        size_t best = 0;
        for (size_t i = 1; i + 1 < ts.size(); ++i)
            if ((double)ts[i] / ts[i + 1] >= (double)ts[best] / ts[best + 1]) best = i;
        ts.erase(ts.begin() + (long)best);
    }
    for (int t = 0; t <= 8; ++t) {
        launch[t] = 0;
        if (t == 0 || !present[t]) continue;
        for (int u : ts)
            if (u >= t) {
                launch[t] = u;
                break;
            }
    }
}

// two U(0,1) doubles of the library's Philox4x32-10 stream (swim_philox.h)
void uniforms2(uint64_t seed, uint32_t stream, uint64_t index, uint32_t draw, double* u)
{
    philox_uniforms2(seed, stream, index, draw, u);
}

void box_muller(double u, double v, double* z0, double* z1)
{
    const double r = std::sqrt(-2.0 * std::log(u));
    *z0 = r * std::cos(2.0 * M_PI * v);
    *z1 = r * std::sin(2.0 * M_PI * v);
}

// weighted mean and covariance (normalized weights) of an n x 3 population
void wcov3(const double* th, const double* w, int64_t n, double mu[3], double S[9])
{
    double ws = 0;
    for (int64_t i = 0; i < n; ++i) ws += w[i];
    for (int d = 0; d < 3; ++d) {
        double m = 0;
        for (int64_t i = 0; i < n; ++i) m += w[i] * th[3 * i + d];
        mu[d] = m / ws;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0;
            for (int64_t i = 0; i < n; ++i) s += w[i] * (th[3 * i + a] - mu[a]) * (th[3 * i + b] - mu[b]);
            S[3 * a + b] = s / ws;
        }
}

bool chol3(const double* A, double* L)
{
    for (int i = 0; i < 9; ++i) L[i] = 0;
    for (int j = 0; j < 3; ++j) {
        double d = A[3 * j + j];
        for (int k = 0; k < j; ++k) d -= L[3 * j + k] * L[3 * j + k];
        if (!(d > 0)) return false;
        L[3 * j + j] = std::sqrt(d);
        for (int i = j + 1; i < 3; ++i) {
            double s = A[3 * i + j];
            for (int k = 0; k < j; ++k) s -= L[3 * i + k] * L[3 * j + k];
            L[3 * i + j] = s / L[3 * j + j];
        }
    }
    return true;
}

template <typename F> void parallel_for(int64_t n, F f)
{
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 1024) nt = 1;
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t a = t * chunk, b = std::min<int64_t>(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([=]() { for (int64_t i = a; i < b; ++i) f(i); });
    }
    for (auto& x : th) x.join();
}

// Per-system constants in the run's precision; FP32 runs also get the FP64
// constants (after the FP32 ones, 16-byte aligned) from which the kernel
// tables are built.
int sysconst_buffers(swim_ctx* c, int32_t dtype, int64_t n_sys, void** sysc, void** sysc64)
{
    if (dtype == SWIM_F32) {
        const size_t a = (size_t)n_sys * sizeof(SysConst<float>);
        TRY(ensure(c, B_SYSC, a + (size_t)n_sys * sizeof(SysConst<double>)));
        *sysc = c->buf[B_SYSC].p;
        *sysc64 = (char*)c->buf[B_SYSC].p + a;
    } else {
        TRY(ensure(c, B_SYSC, (size_t)n_sys * sizeof(SysConst<double>)));
        *sysc = c->buf[B_SYSC].p;
        *sysc64 = nullptr;
    }
    return SWIM_OK;
}

// ------------------------------------------------------------------------
// forward run (shared by swim_forward and abc_step)
// ------------------------------------------------------------------------
int forward_chunk(swim_ctx* c, int32_t dtype, int64_t n_sys, const int32_t* N, const int32_t* nswim,
                  const double* params_dev, const Run& run, void* obs, void* speed, int32_t* status,
                  int32_t* steps_done, hipStream_t st)
{
    if (n_sys == 0) return SWIM_OK;
    std::vector<int64_t> sw_off(n_sys + 1, 0), big_off(n_sys, 0);
    std::vector<int32_t> nsw(n_sys);
    std::vector<int> pts(n_sys);
    int32_t max_big = 0;
    int64_t big_pts = 0;
    std::vector<std::vector<int32_t>> bucket(8);
    std::vector<int64_t> big_list;
    std::vector<int8_t> tpl_of(n_sys);
    bool present[9] = {}, any_big = false;
    for (int64_t s = 0; s < n_sys; ++s) {
        const int p = N[s] * (nswim ? nswim[s] : 1);
        tpl_of[s] = (int8_t)forward_tpl(dtype, N[s], p, run.eps_over_ds);
        if (tpl_of[s] > 0) present[tpl_of[s]] = true;
        else any_big = true;
    }
    int launch_tpl[9];
    merge_buckets(present, any_big, 1 + swim_ctx::N_AUX, launch_tpl);
    if (c->forced_launch)
        for (int t = 0; t <= 8; ++t) launch_tpl[t] = c->force_launch_tpl[t];
    for (int64_t s = 0; s < n_sys; ++s) {
        nsw[s] = nswim ? nswim[s] : 1;
        sw_off[s + 1] = sw_off[s] + nsw[s];
        pts[s] = N[s] * nsw[s];
        const int tpl = tpl_of[s] > 0 ? launch_tpl[tpl_of[s]] : -1;
        if (tpl > 0) {
            bucket[tpl - 1].push_back((int32_t)s);
        } else {
            big_list.push_back(s);
            big_off[s] = big_pts;
            big_pts += pts[s];
            max_big = std::max(max_big, pts[s]);
        }
    }
    // longest-first order inside every bucket; in a merged bucket, the
    // systems merged in from smaller buckets first (each group longest-
    // first): in a launch of their own they would have started at once,
    // and behind the larger group they would start only once all of its
    // systems are taken (in a generation whose large draws mostly blow up,
    // the few long runs are then the last to start)
    std::vector<int32_t> order;
    std::vector<std::pair<int, int64_t>> bucket_span;  // (tpl, start)
    for (int t : TPL_CHOICES) {
        auto& v = bucket[t - 1];
        if (v.empty()) continue;
        std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) {
            return tpl_of[a] != tpl_of[b] ? tpl_of[a] < tpl_of[b] : pts[a] > pts[b];
        });
        bucket_span.push_back({t, (int64_t)order.size()});
        order.insert(order.end(), v.begin(), v.end());
    }
    // large systems: FP32 at the automatic choice takes the symmetric step
    // (tile pairs, then tiles, of 256 points); otherwise target blocks of
    // 256 * tpl_big points of the one-sided step
    const bool big_sym = dtype == SWIM_F32 && c->opt_big_tpl == 0;
    const int tpl_big = c->opt_big_tpl ? c->opt_big_tpl : 1;
    std::vector<int64_t> blk_s, blk_f;
    std::vector<int64_t> bp_sys, bt_sys, bt_poff;
    std::vector<int32_t> bp_tile, bt_tile;
    int64_t bt_slots = 0;
    if (big_sym) {
        // tile pairs: the off-diagonal ones (twice the work) first, so that
        // the launch's tail holds the lighter diagonal ones
        bt_poff.assign(n_sys, 0);
        std::vector<int64_t> dg_sys;
        std::vector<int32_t> dg_tile;
        for (int64_t s : big_list) {
            const int nt = (pts[s] + BIG_TILE_POINTS - 1) / BIG_TILE_POINTS;
            if (nt > 0xFFFF) return fail(SWIM_EINVAL, "system of %d points exceeds the large-system tiling", pts[s]);
            bt_poff[s] = bt_slots;
            bt_slots += (int64_t)nt * nt;
            for (int ta = 0; ta < nt; ++ta) {
                bt_sys.push_back(s);
                bt_tile.push_back(ta);
                dg_sys.push_back(s);
                dg_tile.push_back(ta | (ta << 16));
                for (int tb = ta + 1; tb < nt; ++tb) {
                    bp_sys.push_back(s);
                    bp_tile.push_back(ta | (tb << 16));
                }
            }
        }
        bp_sys.insert(bp_sys.end(), dg_sys.begin(), dg_sys.end());
        bp_tile.insert(bp_tile.end(), dg_tile.begin(), dg_tile.end());
    } else {
        for (int64_t s : big_list)
            for (int64_t f = 0; f < pts[s]; f += 256 * tpl_big) {
                blk_s.push_back(s);
                blk_f.push_back(f);
            }
    }
    const size_t es = dtype == SWIM_F32 ? 4 : 8;
    size_t total = (sw_off.size() + big_off.size() + big_list.size() + 2 * blk_s.size()) * 8 +
                   (nsw.size() + order.size()) * 4 + n_sys * 4 + 64 +
                   (bp_sys.size() + bt_sys.size() + bt_poff.size()) * 8 + (bp_tile.size() + bt_tile.size()) * 4 +
                   6 * 256;
    TRY(begin_uploads(c, total));
    TRY(stage(c, sw_off.data(), sw_off.size() * 8, B_SWOFF, st));
    TRY(stage(c, big_off.data(), big_off.size() * 8, B_OFF, st));
    TRY(stage(c, N, n_sys * 4, B_NPT, st));
    TRY(stage(c, nsw.data(), nsw.size() * 4, B_NSW, st));
    TRY(stage(c, order.data(), order.size() * 4, B_ORDER, st));
    TRY(stage(c, big_list.data(), big_list.size() * 8, B_LIST, st));
    TRY(stage(c, blk_s.data(), blk_s.size() * 8, B_BLKS, st));
    TRY(stage(c, blk_f.data(), blk_f.size() * 8, B_BLKF, st));
    if (big_sym) {
        TRY(stage(c, bp_sys.data(), bp_sys.size() * 8, B_BT_PSYS, st));
        TRY(stage(c, bp_tile.data(), bp_tile.size() * 4, B_BT_PT, st));
        TRY(stage(c, bt_sys.data(), bt_sys.size() * 8, B_BT_TSYS, st));
        TRY(stage(c, bt_tile.data(), bt_tile.size() * 4, B_BT_TT, st));
        TRY(stage(c, bt_poff.data(), bt_poff.size() * 8, B_BT_POFF, st));
    }
    TRY(end_uploads(c, st));
    void *sysc, *sysc64;
    TRY(sysconst_buffers(c, dtype, n_sys, &sysc, &sysc64));
    TRY(ensure(c, B_QUEUE, 8 * 4));
    if (dtype == SWIM_F32) TRY(ensure(c, B_TAB, (size_t)n_sys * table_bytes()));
    Batch b;
    b.n_sys = n_sys;
    b.pt_off = (const int64_t*)c->buf[B_OFF].p;
    b.sw_off = (const int64_t*)c->buf[B_SWOFF].p;
    b.npt = (const int32_t*)c->buf[B_NPT].p;
    b.nswim = (const int32_t*)c->buf[B_NSW].p;
    b.params = params_dev;
    b.sysc = sysc;
    b.sysc64 = sysc64;
    b.tab = dtype == SWIM_F32 ? c->buf[B_TAB].p : nullptr;
    // launch shapes of the persistent buckets (and their LDS limits, set
    // here: nothing inside a stream capture may change them)
    struct Bucket {
        int tpl, wps, nblocks, lane = 0;
        int64_t start, count;
    };
    std::vector<Bucket> bk;
    for (size_t k = 0; k < bucket_span.size(); ++k) {
        Bucket q;
        q.tpl = bucket_span[k].first;
        q.start = bucket_span[k].second;
        q.count = (k + 1 < bucket_span.size() ? bucket_span[k + 1].second : (int64_t)order.size()) - q.start;
        // untuned default: 16 waves, except FP32 systems of 65..128 points,
        // which take 8 (16 offsets of the pair schedule per wave instead of 8
        // halves the per-wave share of each step's fixed work; two systems
        // per CU either way)
        const int wps_default = (dtype == SWIM_F32 && q.tpl == 2) ? 8 : 16;
        q.wps = c->opt_wps ? c->opt_wps : (c->tuned_wps[dtype][q.tpl] ? c->tuned_wps[dtype][q.tpl] : wps_default);
        // at most FWD_MAX_WINDOWS point windows per lane: fewer waves are not
        // built (their one-wave instantiations exceed 256 VGPRs and spill to
        // AGPRs), and an explicit request for them is refused; the wave
        // partial sums of one system must also fit the LDS
        if (c->opt_wps && c->opt_wps < forward_min_wps(q.tpl))
            return fail(SWIM_EINVAL,
                        "SWIM_OPT_WPS = %d is below the %d waves per system needed for systems of up to %d points "
                        "(at most 5 point windows of 60 per lane)",
                        c->opt_wps, forward_min_wps(q.tpl), 64 * q.tpl);
        q.wps = std::max(q.wps, forward_min_wps(q.tpl));
        while (q.wps > forward_min_wps(q.tpl) && forward_lds_bytes(dtype, q.tpl, q.wps) > 160 * 1024) q.wps /= 2;
        const int per_cu = forward_blocks_per_cu(dtype, q.tpl, q.wps);
        q.nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(q.count, (int64_t)per_cu * c->num_cu));
        HIPCHK(prepare_forward(dtype, q.tpl, q.wps));
        bk.push_back(q);
    }
    // lanes of the concurrent launch (longest processing time first): each
    // part, in decreasing pair work, goes to the lane with the least work
    int big_lane = 0;
    {
        const int parts = (int)bk.size() + (big_list.empty() ? 0 : 1);
        const int lanes = std::min(parts, 1 + swim_ctx::N_AUX);
        std::vector<std::pair<double, int>> work;  // (pair work, part: bucket k or -1 for the large systems)
        for (size_t k = 0; k < bk.size(); ++k) {
            double w = 0.0;
            for (int64_t i = bk[k].start; i < bk[k].start + bk[k].count; ++i) w += (double)pts[order[i]] * pts[order[i]];
            work.push_back({w, (int)k});
        }
        if (!big_list.empty()) {
            double w = 0.0;
            for (int64_t s : big_list) w += (double)pts[s] * pts[s];
            work.push_back({w, -1});
        }
        std::stable_sort(work.begin(), work.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
        std::vector<double> load(std::max(lanes, 1), 0.0);
        for (const auto& wk : work) {
            const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[l] += wk.first;
            if (wk.second >= 0) bk[wk.second].lane = l;
            else big_lane = l;
        }
    }
    BigState S{};
    if (!big_list.empty()) {
        const size_t one = (size_t)big_pts * es;
        TRY(ensure(c, B_BIG, 8 * one + sw_off[n_sys] * 2 * es + 256));
        char* base = (char*)c->buf[B_BIG].p;
        for (int q = 0; q < 2; ++q) {
            S.xh[q] = base + (0 + q) * one;
            S.yh[q] = base + (2 + q) * one;
            S.xl[q] = base + (4 + q) * one;
            S.yl[q] = base + (6 + q) * one;
        }
        S.head0 = base + 8 * one;
        if (big_sym) {
            TRY(ensure(c, B_BT_PART, (size_t)bt_slots * BIG_TILE_POINTS * 2 * sizeof(double)));
            HIPCHK(prepare_big_pairs());
        } else {
            if (big_step_lds_bytes(dtype, max_big) > 160 * 1024)
                return fail(SWIM_EINVAL, "system of %d points exceeds the LDS capacity", max_big);
            HIPCHK(prepare_big_step(dtype, tpl_big, max_big));
        }
    }
    BigTiles bt_pairs{}, bt_tiles{};
    if (big_sym) {
        bt_pairs.sys = (const int64_t*)c->buf[B_BT_PSYS].p;
        bt_pairs.tile = (const int32_t*)c->buf[B_BT_PT].p;
        bt_pairs.poff = (const int64_t*)c->buf[B_BT_POFF].p;
        bt_pairs.part = c->buf[B_BT_PART].p;
        bt_tiles = bt_pairs;
        bt_tiles.sys = (const int64_t*)c->buf[B_BT_TSYS].p;
        bt_tiles.tile = (const int32_t*)c->buf[B_BT_TT].p;
    }
    // the launch sequence of the run (uploads above are not part of it)
    auto launch_all = [&]() -> hipError_t {
        hipError_t e = launch_sysconst_batch(dtype, n_sys, (const int64_t*)c->buf[B_SWOFF].p,
                                             (const int32_t*)c->buf[B_NPT].p, params_dev, run.eps_over_ds, sysc,
                                             sysc64, status, c->opt_blob, st);
        if (e == hipSuccess && dtype == SWIM_F32) e = launch_table_build(0, n_sys, sysc64, c->buf[B_TAB].p, c->opt_blob, st);
        if (e == hipSuccess) e = launch_fill_i32((int32_t*)c->buf[B_QUEUE].p, 0, 8, st);
        if (e == hipSuccess && c->opt_time) e = hipEventRecord(c->time_ev[0], st);
        // Buckets (and the large systems) are independent: with more than
        // one, they run side by side, the call's stream and up to N_AUX
        // auxiliary streams each taking a share (lanes assigned in order of
        // decreasing work), forked from the set-up above and joined before
        // the call returns, so that one bucket's tail overlaps the others.
        const int parts = (int)bk.size() + (big_list.empty() ? 0 : 1);
        const int lanes = std::min(parts, 1 + swim_ctx::N_AUX);
        auto lane_stream = [&](int l) { return l == 0 ? st : c->aux[l - 1]; };
        if (e == hipSuccess && lanes > 1) {
            e = hipEventRecord(c->fork_ev, st);
            for (int l = 1; l < lanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(c->aux[l - 1], c->fork_ev, 0);
        }
        for (size_t k = 0; k < bk.size() && e == hipSuccess; ++k) {
            Batch bb = b;
            bb.n_sys = bk[k].count;
            e = launch_forward(dtype, bk[k].tpl, bk[k].wps, bk[k].nblocks, bb, run,
                               (const int32_t*)c->buf[B_ORDER].p + bk[k].start, (int32_t*)c->buf[B_QUEUE].p + k, obs,
                               speed, status, steps_done, lane_stream(bk[k].lane % lanes));
        }
        if (!big_list.empty() && e == hipSuccess) {
            const hipStream_t st_big = lane_stream(big_lane % lanes);
            e = launch_big_init(dtype, (const int64_t*)c->buf[B_LIST].p, (int64_t)big_list.size(), b, S, status, obs,
                                run.n_obs, st_big);
            for (int step = 0; step < run.steps && e == hipSuccess; ++step) {
                if (big_sym) {
                    e = launch_big_pairs((int64_t)bp_sys.size(), bt_pairs, b, S, step, run, status, st_big);
                    if (e == hipSuccess)
                        e = launch_big_update((int64_t)bt_sys.size(), bt_tiles, b, S, step, run, obs, status,
                                              steps_done, st_big);
                } else {
                    e = launch_big_step(dtype, tpl_big, (int64_t)blk_s.size(), (const int64_t*)c->buf[B_BLKS].p,
                                        (const int64_t*)c->buf[B_BLKF].p, max_big, b, S, step, run, obs, status,
                                        steps_done, st_big);
                }
            }
            if (e == hipSuccess)
                e = launch_big_finish(dtype, (const int64_t*)c->buf[B_LIST].p, (int64_t)big_list.size(), b, S,
                                      run.steps & 1, run, speed, status, steps_done, st_big);
        }
        for (int l = 1; l < lanes && e == hipSuccess; ++l) {
            e = hipEventRecord(c->join_ev[l - 1], c->aux[l - 1]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, c->join_ev[l - 1], 0);
        }
        if (e == hipSuccess && c->opt_time) e = hipEventRecord(c->time_ev[1], st);
        return e;
    };
    if (c->opt_graph == 0 || c->opt_time) {
        // timed calls launch eagerly: the events stay plain stream events
        c->timed = false;
        HIPCHK(launch_all());
        c->timed = c->opt_time != 0;
        return SWIM_OK;
    }
    // key of the layout: everything the launch sequence bakes in
    Fnv h;
    h.add(dtype);
    h.add(n_sys);
    h.add_bytes(N, (size_t)n_sys * 4);
    h.add_bytes(nsw.data(), nsw.size() * 4);
    h.add(run.steps);
    h.add(run.dt);
    h.add(run.obs_every);
    h.add(run.n_obs);
    h.add(run.eps_over_ds);
    h.add(run.stop_data);
    h.add(run.stop_ssq);
    h.add(tpl_big);
    h.add(big_sym ? 1 : 0);
    h.add(c->opt_blob);
    for (const Bucket& q : bk) {
        h.add(q.tpl);
        h.add(q.wps);
        h.add(q.nblocks);
        h.add(q.lane);
    }
    h.add(big_lane);
    const void* ptrs[] = {params_dev, obs, speed, status, steps_done, sysc, sysc64, b.tab, c->buf[B_SWOFF].p,
                          c->buf[B_OFF].p, c->buf[B_NPT].p, c->buf[B_NSW].p, c->buf[B_ORDER].p, c->buf[B_LIST].p,
                          c->buf[B_QUEUE].p, c->buf[B_BIG].p, st};
    h.add_bytes(ptrs, sizeof(ptrs));
    // the large-system step's own lists: only those its launches read (the
    // other path's buffers are shared with other calls, which may move them)
    if (!big_list.empty()) {
        const void* bptrs[] = {c->buf[B_BLKS].p, c->buf[B_BLKF].p};
        const void* sptrs[] = {c->buf[B_BT_PSYS].p, c->buf[B_BT_PT].p, c->buf[B_BT_TSYS].p,
                               c->buf[B_BT_TT].p,   c->buf[B_BT_POFF].p, c->buf[B_BT_PART].p};
        if (big_sym)
            h.add_bytes(sptrs, sizeof(sptrs));
        else
            h.add_bytes(bptrs, sizeof(bptrs));
    }
    const uint64_t key = h.v;
    ++c->graph_clock;
    for (auto& g : c->graphs)
        if (g.exec && g.key == key) {
            g.last_use = c->graph_clock;
            HIPCHK(hipGraphLaunch(g.exec, st));
            ++c->graph_launches;
            return SWIM_OK;
        }
    if (c->opt_graph == 1 && key != c->last_key) {
        // first sight of this layout: run eagerly, capture if it recurs
        c->last_key = key;
        HIPCHK(launch_all());
        return SWIM_OK;
    }
    // capture into the least recently used slot
    FwdGraph* slot = &c->graphs[0];
    for (auto& g : c->graphs)
        if (!g.exec || g.last_use < slot->last_use) slot = &g;
    if (slot->exec) HIPCHK(hipGraphExecDestroy(slot->exec));
    if (slot->graph) HIPCHK(hipGraphDestroy(slot->graph));
    slot->exec = nullptr;
    slot->graph = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const hipError_t le = launch_all();
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(st, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return fail(SWIM_EHIP, "capture of the forward run failed: %s", hipGetErrorString(le != hipSuccess ? le : ce));
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return fail(SWIM_EHIP, "instantiation of the forward-run graph failed");
    }
    slot->graph = graph;
    slot->exec = exec;
    slot->key = key;
    slot->last_use = c->graph_clock;
    c->last_key = key;
    ++c->graph_captures;
    HIPCHK(hipGraphLaunch(exec, st));
    ++c->graph_launches;
    return SWIM_OK;
}


// FP32 runs keep one kernel table per system in HBM (12 KB each), so very
// large batches run in chunks of FWD_CHUNK systems; the systems are
// independent and their order within a batch does not change any result.
constexpr int64_t FWD_CHUNK = 262144;

int forward_impl(swim_ctx* c, int32_t dtype, int64_t n_sys, const int32_t* N, const int32_t* nswim,
                 const double* params_dev, const Run& run, void* obs, void* speed, int32_t* status,
                 int32_t* steps_done, hipStream_t st)
{
    if (dtype != SWIM_F32 || n_sys <= FWD_CHUNK)
        return forward_chunk(c, dtype, n_sys, N, nswim, params_dev, run, obs, speed, status, steps_done, st);
    const size_t es = 4;
    int64_t f0 = 0;  // first filament of the chunk
    for (int64_t s0 = 0; s0 < n_sys; s0 += FWD_CHUNK) {
        const int64_t m = std::min(FWD_CHUNK, n_sys - s0);
        int64_t nf = 0;
        for (int64_t s = s0; s < s0 + m; ++s) nf += nswim ? nswim[s] : 1;
        TRY(forward_chunk(c, dtype, m, N + s0, nswim ? nswim + s0 : nullptr, params_dev + f0 * SWIM_NPARAM, run,
                          (char*)obs + (size_t)f0 * run.n_obs * 2 * es, (char*)speed + (size_t)f0 * es, status + s0,
                          steps_done ? steps_done + s0 : nullptr, st));
        f0 += nf;
    }
    return SWIM_OK;
}

// ------------------------------------------------------------------------
// surrogate MLP: forward and backward over M rows (workspace in the ctx)
// activation workspace layout (floats): pre[4][M*256], H[4][M*256],
// Y[M*33], dY[M*33], dA[2][M*256], rowsq[M]
// ------------------------------------------------------------------------
struct MlpAct {
    float* pre[4];
    float* H[4];
    float *Y, *dY, *dA[2], *sq;
    MlpWs ws;  // split-K partial sums of the GEMMs
};

int mlp_act(swim_ctx* c, int64_t M, MlpAct* a)
{
    const int64_t H = 256, O = 33;
    const int64_t ws = 1 << 20;  // partial sums: 16 slices of 256 x 256, or 4 of 1024 x 256
    const int64_t total = 8 * M * H + 2 * M * O + 2 * M * H + M * O + ws;
    TRY(ensure(c, B_MLP_ACT, (size_t)total * 4));
    float* p = (float*)c->buf[B_MLP_ACT].p;
    for (int l = 0; l < 4; ++l) a->pre[l] = p + l * M * H;
    for (int l = 0; l < 4; ++l) a->H[l] = p + (4 + l) * M * H;
    a->Y = p + 8 * M * H;
    a->dY = a->Y + M * O;
    a->dA[0] = a->dY + M * O;
    a->dA[1] = a->dA[0] + M * H;
    a->sq = a->dA[1] + M * H;
    a->ws.part = a->sq + M * O;
    a->ws.part_floats = ws;
    return SWIM_OK;
}

// forward pass; with T (training), the output layer's epilogue also forms
// the gradient of the squared error, dY = 2 (Y - T) / (M 33), and the
// squared errors (a.dY, a.sq)
int mlp_forward(const float* X, const float* P, int64_t M, const MlpAct& a, float* Y, hipStream_t st,
                const float* T = nullptr)
{
    const float* in = X;
    int64_t ldin = MLP_W[0];
    for (int l = 0; l < MLP_L; ++l) {
        const int K = MLP_W[l], N = MLP_W[l + 1];
        const float* W = P + mlp_offW(l);
        GemmEpi E;
        E.bias = P + mlp_offb(l);
        if (l < MLP_L - 1) {
            E.aux = a.H[l];
            HIPCHK(launch_gemm_bf16(1, (int)M, N, K, in, ldin, 1, W, N, 1, a.pre[l], N, E, a.ws, st));
            in = a.H[l];
            ldin = N;
        } else if (T) {
            E.aux = a.dY;
            E.T = T;
            E.sq = a.sq;
            E.sc = 2.0f / ((float)M * (float)N);
            HIPCHK(launch_gemm_bf16(4, (int)M, N, K, in, ldin, 1, W, N, 1, Y, N, E, a.ws, st));
        } else {
            HIPCHK(launch_gemm_bf16(2, (int)M, N, K, in, ldin, 1, W, N, 1, Y, N, E, a.ws, st));
        }
    }
    return SWIM_OK;
}

// gradients of the squared error into G (layout of the parameters), after
// mlp_forward with the targets; loss (device, optional) = the sum of the
// M x 33 squared errors
int mlp_backward(const float* X, const float* P, int64_t M, const MlpAct& a, float* G, float* loss, hipStream_t st)
{
    const int O = MLP_W[MLP_L];
    if (loss) HIPCHK(launch_sum(M * O, a.sq, loss, st));
    const float* dA = a.dY;
    int cur = 0;
    for (int l = MLP_L - 1; l >= 0; --l) {
        const int K = MLP_W[l], N = MLP_W[l + 1];
        const float* Hin = l > 0 ? a.H[l - 1] : X;
        // dW_l = Hin^T dA  (K x N, summed over the M rows)
        HIPCHK(launch_gemm_bf16(0, K, N, (int)M, Hin, 1, K, dA, N, 1, G + mlp_offW(l), N, GemmEpi(), a.ws, st));
        HIPCHK(launch_colsum((int)M, N, dA, N, G + mlp_offb(l), st));
        if (l > 0) {
            // dA_{l-1} = (dA W_l^T) * gelu'(pre_{l-1})
            float* out = a.dA[cur];
            GemmEpi E;
            E.aux = a.pre[l - 1];
            HIPCHK(launch_gemm_bf16(3, (int)M, K, N, dA, N, 1, P + mlp_offW(l), 1, N, out, K, E, a.ws, st));
            dA = out;
            cur ^= 1;
        }
    }
    return SWIM_OK;
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char* swim_last_error(void) { return g_err.c_str(); }

int swim_version(void) { return 1; }

int swim_create(swim_ctx** out, int device)
{
    if (!out) return fail(SWIM_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(SWIM_EINVAL, "device %d out of range (%d devices)", device, n);
    HIPCHK(hipSetDevice(device));
    swim_ctx* c = new swim_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess || hipStreamCreateWithFlags(&c->stream, hipStreamDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->up_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->sw_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->time_ev[0], hipEventDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->time_ev[1], hipEventDefault) != hipSuccess) {
        (void)hipGetLastError();
        swim_destroy(c);
        return fail(SWIM_EHIP, "context creation failed");
    }
    c->num_cu = prop.multiProcessorCount;
    for (int k = 0; k < swim_ctx::N_AUX; ++k) {
        if (hipStreamCreateWithFlags(&c->aux[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->join_ev[k], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            swim_destroy(c);
            return fail(SWIM_EHIP, "context creation failed (auxiliary streams)");
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (device < NOALLOC_MAX_DEV && !g_scratch_dev[device]) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                swim_destroy(c);
                return fail(SWIM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            }
            g_scratch_dev[device] = p;
        }
    }
    *out = c;
    return SWIM_OK;
}

void swim_destroy(swim_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& b : c->buf)
        if (b.p) (void)hipFree(b.p);
    for (auto& g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->up_ev) (void)hipEventDestroy(c->up_ev);
    if (c->sw_ev) (void)hipEventDestroy(c->sw_ev);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    for (auto& ev : c->time_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (int k = 0; k < swim_ctx::N_AUX; ++k) {
        if (c->aux[k]) {
            (void)hipStreamSynchronize(c->aux[k]);
            (void)hipStreamDestroy(c->aux[k]);
        }
        if (c->join_ev[k]) (void)hipEventDestroy(c->join_ev[k]);
    }
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int swim_set_option(swim_ctx* c, int32_t key, int32_t value)
{
    if (!c) return fail(SWIM_EINVAL, "null context");
    if (key == SWIM_OPT_WPS) {
        if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
            return fail(SWIM_EINVAL, "waves per system must be 0, 1, 2, 4, 8 or 16");
        c->opt_wps = value;
    } else if (key == SWIM_OPT_BIG_TPL) {
        if (value != 0 && value != 1 && value != 2 && value != 4) return fail(SWIM_EINVAL, "targets per lane must be 0, 1, 2 or 4");
        c->opt_big_tpl = value;
    } else if (key == SWIM_OPT_GRAPH) {
        if (value < 0 || value > 2) return fail(SWIM_EINVAL, "graph mode must be 0, 1 or 2");
        c->opt_graph = value;
    } else if (key == SWIM_OPT_BLOB) {
        if (value != SWIM_BLOB_READING && value != SWIM_BLOB_PAPER) return fail(SWIM_EINVAL, "blob must be 0 or 1");
        c->opt_blob = value;
    } else if (key == SWIM_OPT_EARLY_STOP) {
        if (value != 0 && value != 1) return fail(SWIM_EINVAL, "early stop must be 0 or 1");
        c->opt_early_stop = value;
    } else if (key == SWIM_OPT_TIME_KERNEL) {
        if (value != 0 && value != 1) return fail(SWIM_EINVAL, "kernel timing must be 0 or 1");
        c->opt_time = value;
        c->timed = false;
    } else {
        return fail(SWIM_EINVAL, "unknown option %d", key);
    }
    return SWIM_OK;
}

int swim_get_option(swim_ctx* c, int32_t key, int32_t* value)
{
    if (!c || !value) return fail(SWIM_EINVAL, "null argument");
    if (key == SWIM_OPT_WPS) *value = c->opt_wps;
    else if (key == SWIM_OPT_BIG_TPL) *value = c->opt_big_tpl;
    else if (key == SWIM_OPT_GRAPH) *value = c->opt_graph;
    else if (key == SWIM_OPT_BLOB) *value = c->opt_blob;
    else if (key == SWIM_OPT_EARLY_STOP) *value = c->opt_early_stop;
    else if (key == SWIM_OPT_TIME_KERNEL) *value = c->opt_time;
    else if (key == SWIM_OPT_KERNEL_US) {
        if (!c->timed) return fail(SWIM_ESTATE, "no timed forward call (set SWIM_OPT_TIME_KERNEL first)");
        (void)hipSetDevice(c->device);
        float ms = 0.0f;
        HIPCHK(hipEventSynchronize(c->time_ev[1]));
        HIPCHK(hipEventElapsedTime(&ms, c->time_ev[0], c->time_ev[1]));
        *value = (int32_t)std::min(2.0e9, std::round(1e3 * (double)ms));
    }
    else if (key == SWIM_OPT_GRAPH_LAUNCHES) *value = (int32_t)c->graph_launches;
    else if (key == SWIM_OPT_GRAPH_CAPTURES) *value = (int32_t)c->graph_captures;
    else return fail(SWIM_EINVAL, "unknown option %d", key);
    return SWIM_OK;
}

int swim_pair_velocity(swim_ctx* c, int32_t dtype, int64_t n_sys, const int64_t* sys_off, const double* alpha,
                       const double* eps, const void* x, const void* y, const void* fx, const void* fy, void* ux,
                       void* uy, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n_sys < 0) return fail(SWIM_EINVAL, "n_sys < 0");
    if (n_sys == 0) return SWIM_OK;
    if (!sys_off || !alpha || !eps) return fail(SWIM_EINVAL, "sys_off/alpha/eps must be host arrays");
    if (sys_off[0] != 0) return fail(SWIM_EINVAL, "sys_off[0] must be 0");
    for (int64_t s = 0; s < n_sys; ++s) {
        if (sys_off[s + 1] < sys_off[s]) return fail(SWIM_EINVAL, "sys_off must be non-decreasing (system %lld)", (long long)s);
        if (!(std::isfinite(alpha[s]) && alpha[s] >= 0)) return fail(SWIM_EINVAL, "alpha[%lld] must be finite and >= 0", (long long)s);
        if (!(std::isfinite(eps[s]) && eps[s] > 0)) return fail(SWIM_EINVAL, "eps[%lld] must be finite and > 0", (long long)s);
        if (alpha[s] * eps[s] > 1.0) return fail(SWIM_EINVAL, "alpha*eps > 1 for system %lld", (long long)s);
    }
    const int64_t npts = sys_off[n_sys];
    if (npts > 0 && (!x || !y || !fx || !fy || !ux || !uy)) return fail(SWIM_EINVAL, "null data pointer");
    hipStream_t st = pick(c, stream);
    int64_t maxn = 0;
    for (int64_t s = 0; s < n_sys; ++s) maxn = std::max(maxn, sys_off[s + 1] - sys_off[s]);
    const int tpl = maxn >= 2048 ? 2 : 1;
    std::vector<int64_t> bs, bf;
    for (int64_t s = 0; s < n_sys; ++s)
        for (int64_t f = 0; f < sys_off[s + 1] - sys_off[s]; f += 256 * tpl) {
            bs.push_back(s);
            bf.push_back(f);
        }
    TRY(begin_uploads(c, (n_sys + 1) * 8 + 2 * n_sys * 8 + 2 * bs.size() * 8));
    TRY(stage(c, sys_off, (n_sys + 1) * 8, B_OFF, st));
    TRY(stage(c, alpha, n_sys * 8, B_ALPHA, st));
    TRY(stage(c, eps, n_sys * 8, B_EPS, st));
    TRY(stage(c, bs.data(), bs.size() * 8, B_BLKS, st));
    TRY(stage(c, bf.data(), bf.size() * 8, B_BLKF, st));
    TRY(end_uploads(c, st));
    void *sysc, *sysc64;
    TRY(sysconst_buffers(c, dtype, n_sys, &sysc, &sysc64));
    HIPCHK(launch_sysconst(dtype, n_sys, (const double*)c->buf[B_ALPHA].p, (const double*)c->buf[B_EPS].p, sysc,
                           sysc64, c->opt_blob, st));
    void* tab = nullptr;
    if (dtype == SWIM_F32) {
        TRY(ensure(c, B_TAB, (size_t)n_sys * table_bytes()));
        HIPCHK(launch_table_build(0, n_sys, sysc64, c->buf[B_TAB].p, c->opt_blob, st));
        tab = c->buf[B_TAB].p;
    }
    HIPCHK(launch_pair_velocity(dtype, tpl, (int64_t)bs.size(), (const int64_t*)c->buf[B_BLKS].p,
                                (const int64_t*)c->buf[B_BLKF].p, (const int64_t*)c->buf[B_OFF].p, sysc, tab, x, y,
                                fx, fy, ux, uy, st));
    return SWIM_OK;
}

int swim_pair_velocity_noalloc(swim_ctx* c, int32_t dtype, int64_t n_sys, const int64_t* sys_off,
                               const double* alpha, const double* eps, const void* x, const void* y, const void* fx,
                               const void* fy, void* ux, void* uy, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n_sys < 0) return fail(SWIM_EINVAL, "n_sys < 0");
    if (n_sys == 0) return SWIM_OK;
    if (n_sys > NOALLOC_MAX_SYS)
        return fail(SWIM_EINVAL, "n_sys = %lld exceeds the no-allocation workspace (%lld systems)", (long long)n_sys,
                    (long long)NOALLOC_MAX_SYS);
    if (!sys_off || !alpha || !eps) return fail(SWIM_EINVAL, "sys_off/alpha/eps must be host arrays");
    if (sys_off[0] != 0) return fail(SWIM_EINVAL, "sys_off[0] must be 0");
    for (int64_t s = 0; s < n_sys; ++s) {
        if (sys_off[s + 1] < sys_off[s]) return fail(SWIM_EINVAL, "sys_off must be non-decreasing (system %lld)", (long long)s);
        if (!(std::isfinite(alpha[s]) && alpha[s] >= 0)) return fail(SWIM_EINVAL, "alpha[%lld] must be finite and >= 0", (long long)s);
        if (!(std::isfinite(eps[s]) && eps[s] > 0)) return fail(SWIM_EINVAL, "eps[%lld] must be finite and > 0", (long long)s);
        if (alpha[s] * eps[s] > 1.0) return fail(SWIM_EINVAL, "alpha*eps > 1 for system %lld", (long long)s);
    }
    const int64_t npts = sys_off[n_sys];
    if (npts > 0 && (!x || !y || !fx || !fy || !ux || !uy)) return fail(SWIM_EINVAL, "null data pointer");
    if (c->device >= NOALLOC_MAX_DEV || !g_scratch_dev[c->device])
        return fail(SWIM_ESTATE, "no workspace address for device %d", c->device);
    char* ws = (char*)g_scratch_dev[c->device];
    int64_t maxn = 0;
    for (int64_t s = 0; s < n_sys; ++s) maxn = std::max(maxn, sys_off[s + 1] - sys_off[s]);
    const int tpl = maxn >= 2048 ? 2 : 1;
    int64_t nb = 0;
    for (int64_t s = 0; s < n_sys; ++s) nb += (sys_off[s + 1] - sys_off[s] + 256 * tpl - 1) / (256 * tpl);
    if (nb > NOALLOC_MAX_BLOCKS)
        return fail(SWIM_EINVAL, "%lld pair-kernel blocks exceed the no-allocation workspace (%lld)", (long long)nb,
                    (long long)NOALLOC_MAX_BLOCKS);
    // the host data of the call, laid out as in the workspace, on the stack;
    // one synchronous copy on the stream (no pinned staging buffer)
    alignas(16) unsigned char host[NA_SYSC];
    memcpy(host + NA_OFF, sys_off, (size_t)(n_sys + 1) * 8);
    memcpy(host + NA_ALPHA, alpha, (size_t)n_sys * 8);
    memcpy(host + NA_EPS, eps, (size_t)n_sys * 8);
    int64_t* bs = (int64_t*)(host + NA_BLKS);
    int64_t* bf = (int64_t*)(host + NA_BLKF);
    int64_t k = 0;
    for (int64_t s = 0; s < n_sys; ++s)
        for (int64_t f = 0; f < sys_off[s + 1] - sys_off[s]; f += 256 * tpl) {
            bs[k] = s;
            bf[k] = f;
            ++k;
        }
    hipStream_t st = pick(c, stream);
    HIPCHK(hipMemcpyWithStream(ws, host, NA_SYSC, hipMemcpyHostToDevice, st));
    void* sysc = ws + NA_SYSC;
    void* sysc64 = dtype == SWIM_F32 ? (void*)(ws + NA_SYSC64) : nullptr;
    HIPCHK(launch_sysconst(dtype, n_sys, (const double*)(ws + NA_ALPHA), (const double*)(ws + NA_EPS), sysc, sysc64,
                           c->opt_blob, st));
    void* tab = nullptr;
    if (dtype == SWIM_F32) {
        tab = ws + NA_TAB;
        HIPCHK(launch_table_build(0, n_sys, sysc64, tab, c->opt_blob, st));
    }
    HIPCHK(launch_pair_velocity(dtype, tpl, nb, (const int64_t*)(ws + NA_BLKS), (const int64_t*)(ws + NA_BLKF),
                                (const int64_t*)(ws + NA_OFF), sysc, tab, x, y, fx, fy, ux, uy, st));
    return SWIM_OK;
}

int swim_flow_field(swim_ctx* c, int32_t dtype, int64_t n, const void* x, const void* y, const void* fx,
                    const void* fy, double alpha, double eps, int64_t nt, const void* tx, const void* ty, void* u,
                    void* v, void* p, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n < 0 || nt < 0) return fail(SWIM_EINVAL, "negative size");
    if (!(std::isfinite(alpha) && alpha >= 0 && std::isfinite(eps) && eps > 0 && alpha * eps <= 1.0))
        return fail(SWIM_EINVAL, "need alpha >= 0, eps > 0, alpha*eps <= 1");
    if (nt == 0) return SWIM_OK;
    if ((n > 0 && (!x || !y || !fx || !fy)) || !tx || !ty || !u || !v || !p)
        return fail(SWIM_EINVAL, "null device pointer");
    FieldConst fc{};
    sysconst_compute<float>(alpha, eps, &fc.c32, c->opt_blob);
    sysconst_compute<double>(alpha, eps, &fc.c64, c->opt_blob);
    fc.paper = c->opt_blob == SWIM_BLOB_PAPER;
    fc.h1c = fc.c64.h1c;
    fc.e2 = eps * eps;
    fc.inv_e2 = 1.0 / fc.e2;
    fc.eps = eps;
    fc.alpha = alpha;
    fc.inv_2pi = 0.5 / M_PI;
    fc.stokes = alpha == 0.0;
    if (!fc.stokes) {
        // near-contact series of w = m / (2 pi r^2) from g = sum_n gam_n delta^n,
        // gam_n = -(c/2pi) (-1)^n kap_n, kap_n = (z0/2)^n K_n(z0) / n!,
        // c = 1/(z0 K1(z0)): w = (1/eps^2) sum_n [2 (n+1) gam_{n+1}
        // - (alpha^2 eps^2 / 2) gam_n / (n+1)] delta^n
        const double z0 = alpha * eps;
        double K0, K1, Q;
        bessel_k01_q_f64(z0, &K0, &K1, &Q);
        fc.K1e = K1;
        const double cc = 1.0 / (z0 * K1);
        double kap[FIELD_NSER + 1], gam[FIELD_NSER + 1];
        kap[0] = K0;
        kap[1] = 0.5 * z0 * K1;
        for (int k = 1; k < FIELD_NSER; ++k)
            kap[k + 1] = 0.25 * z0 * z0 * kap[k - 1] / ((double)k * (k + 1)) + (double)k * kap[k] / (k + 1);
        for (int k = 0; k <= FIELD_NSER; ++k) gam[k] = -(cc * fc.inv_2pi) * ((k % 2) ? -1.0 : 1.0) * kap[k];
        for (int k = 0; k < FIELD_NSER; ++k)
            fc.ser[k] = fc.inv_e2 * (2.0 * (k + 1) * gam[k + 1] - 0.5 * z0 * z0 * gam[k] / (k + 1));
    }
    hipStream_t st = pick(c, stream);
    const void* tab = nullptr;
    void* wtab = nullptr;
    if (dtype == SWIM_F32) {
        // FP32: the pair kernel from the system's table, as in the forward
        // runs (built on the device from the FP64 kernel functions; for the
        // paper's blob at alpha > 0 from its quadrature)
        TRY(begin_uploads(c, 16));
        TRY(stage(c, &alpha, 8, B_ALPHA, st));
        TRY(stage(c, &eps, 8, B_EPS, st));
        TRY(end_uploads(c, st));
        void *sysc, *sysc64;
        TRY(sysconst_buffers(c, SWIM_F32, 1, &sysc, &sysc64));
        HIPCHK(launch_sysconst(SWIM_F32, 1, (const double*)c->buf[B_ALPHA].p, (const double*)c->buf[B_EPS].p, sysc,
                               sysc64, c->opt_blob, st));
        TRY(ensure(c, B_TAB, table_bytes()));
        HIPCHK(launch_table_build(0, 1, sysc64, c->buf[B_TAB].p, c->opt_blob, st));
        tab = c->buf[B_TAB].p;
        // and the pressure weight's table on the same intervals
        TRY(ensure(c, B_WTAB, (size_t)TAB_N * 16));
        wtab = c->buf[B_WTAB].p;
    }
    HIPCHK(launch_flow_field(dtype, n, x, y, fx, fy, fc, nt, tx, ty, u, v, p, tab, wtab, st));
    return SWIM_OK;
}

int swim_elastic_forces(swim_ctx* c, int32_t dtype, int64_t n_fil, const int32_t* N, const double* params, double t,
                        const void* x, const void* y, void* fx, void* fy, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n_fil < 0) return fail(SWIM_EINVAL, "n_fil < 0");
    if (n_fil == 0) return SWIM_OK;
    if (!N || !params) return fail(SWIM_EINVAL, "N/params must be host arrays");
    if (!std::isfinite(t)) return fail(SWIM_EINVAL, "t must be finite");
    std::vector<int64_t> off(n_fil + 1, 0);
    for (int64_t f = 0; f < n_fil; ++f) {
        if (N[f] < 3 || N[f] > 4096) return fail(SWIM_EINVAL, "N[%lld] = %d outside [3, 4096]", (long long)f, N[f]);
        for (int k = 0; k < SWIM_NPARAM; ++k)
            if (!std::isfinite(params[SWIM_NPARAM * f + k])) return fail(SWIM_EINVAL, "non-finite parameter in row %lld", (long long)f);
        off[f + 1] = off[f] + N[f];
    }
    if (!x || !y || !fx || !fy) return fail(SWIM_EINVAL, "null data pointer");
    hipStream_t st = pick(c, stream);
    TRY(begin_uploads(c, (n_fil + 1) * 8 + n_fil * 4 + n_fil * SWIM_NPARAM * 8));
    TRY(stage(c, off.data(), off.size() * 8, B_OFF, st));
    TRY(stage(c, N, n_fil * 4, B_NPT, st));
    TRY(stage(c, params, n_fil * SWIM_NPARAM * 8, B_PARAMS, st));
    TRY(end_uploads(c, st));
    HIPCHK(launch_forces(dtype, n_fil, (const int64_t*)c->buf[B_OFF].p, (const int32_t*)c->buf[B_NPT].p,
                         (const double*)c->buf[B_PARAMS].p, t, x, y, fx, fy, st));
    return SWIM_OK;
}

static int check_run(int64_t n_sys, const int32_t* N, const int32_t* n_swim, int32_t steps, double dt, int32_t obs_every,
                     double eps_over_ds)
{
    if (n_sys < 0) return fail(SWIM_EINVAL, "n_sys < 0");
    if (n_sys > 0 && !N) return fail(SWIM_EINVAL, "N must be a host array");
    if (steps < 1) return fail(SWIM_EINVAL, "steps must be >= 1");
    if (!(std::isfinite(dt) && dt > 0)) return fail(SWIM_EINVAL, "dt must be finite and > 0");
    if (obs_every < 0) return fail(SWIM_EINVAL, "obs_every must be >= 0");
    if (!(std::isfinite(eps_over_ds) && eps_over_ds > 0)) return fail(SWIM_EINVAL, "eps_over_ds must be finite and > 0");
    for (int64_t s = 0; s < n_sys; ++s) {
        const int ns = n_swim ? n_swim[s] : 1;
        if (N[s] < 3 || N[s] > 4096) return fail(SWIM_EINVAL, "N[%lld] = %d outside [3, 4096]", (long long)s, N[s]);
        if (ns < 1) return fail(SWIM_EINVAL, "n_swim[%lld] must be >= 1", (long long)s);
        if ((int64_t)N[s] * ns > 4096) return fail(SWIM_EINVAL, "system %lld has more than 4096 points", (long long)s);
    }
    return SWIM_OK;
}

int swim_forward(swim_ctx* c, int32_t dtype, int64_t n_sys, const int32_t* N, const int32_t* n_swim,
                 const double* params, int32_t steps, double dt, int32_t obs_every, double eps_over_ds, void* obs,
                 void* speed, int32_t* status, int32_t* steps_done, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    TRY(check_run(n_sys, N, n_swim, steps, dt, obs_every, eps_over_ds));
    if (n_sys == 0) return SWIM_OK;
    if (!params || !speed || !status || (obs_every > 0 && !obs)) return fail(SWIM_EINVAL, "null device pointer");
    Run r;
    r.steps = steps;
    r.dt = dt;
    r.obs_every = obs_every;
    r.n_obs = obs_every > 0 ? steps / obs_every : 0;
    r.eps_over_ds = eps_over_ds;
    return forward_impl(c, dtype, n_sys, N, n_swim, params, r, obs, speed, status, steps_done, pick(c, stream));
}

}  // extern "C"

namespace {

int sperm_check(const swim_sperm_shape* shape, int32_t steps, double dt, int32_t obs_every)
{
    if (!shape) return fail(SWIM_EINVAL, "null shape");
    const swim_sperm_shape& sh = *shape;
    if (sh.n_flag < 4) return fail(SWIM_EINVAL, "n_flag must be >= 4");
    if (sh.n_head < 4 || sh.n_head % 2) return fail(SWIM_EINVAL, "n_head must be even and >= 4");
    if (sh.n_swim < 1) return fail(SWIM_EINVAL, "n_swim must be >= 1");
    if ((int64_t)sh.n_swim * (sh.n_flag + sh.n_head) > 512)
        return fail(SWIM_EINVAL, "n_swim * (n_flag + n_head) must be <= 512");
    if (!(std::isfinite(sh.eps) && sh.eps > 0)) return fail(SWIM_EINVAL, "eps must be finite and > 0");
    if (!(std::isfinite(sh.head_radius) && sh.head_radius > 0)) return fail(SWIM_EINVAL, "head_radius must be > 0");
    if (!(std::isfinite(sh.neck_gap) && sh.neck_gap > 0)) return fail(SWIM_EINVAL, "neck_gap must be > 0");
    if (steps < 1) return fail(SWIM_EINVAL, "steps must be >= 1");
    if (!(std::isfinite(dt) && dt > 0)) return fail(SWIM_EINVAL, "dt must be finite and > 0");
    if (obs_every < 0) return fail(SWIM_EINVAL, "obs_every must be >= 0");
    return SWIM_OK;
}

// geometry constants of a (checked) shape
SpermShape sperm_geometry(const swim_sperm_shape& sh)
{
    SpermShape g{};
    g.nf = sh.n_flag;
    g.nh = sh.n_head;
    g.nsw = sh.n_swim;
    g.ds = 1.0 / (double)(sh.n_flag - 1);
    g.hr = sh.head_radius;
    g.dn = sh.neck_gap;
    g.dth = 2.0 * M_PI / (double)sh.n_head;
    g.ch = 2.0 * sh.head_radius * std::sin(0.5 * g.dth);
    g.eps = sh.eps;
    // neck rest lengths from the initial geometry (first flagellum point at
    // the origin)
    const double xf1 = (double)(sh.n_flag - 1) * g.ds, xf2 = (double)(sh.n_flag - 2) * g.ds;
    const double xc = xf1 + g.hr + g.dn;
    const int c0 = sh.n_head / 2;
    auto hx = [&](int m) { return xc + g.hr * std::cos((double)m * g.dth); };
    auto hy = [&](int m) { return g.hr * std::sin((double)m * g.dth); };
    g.L0[0] = std::hypot(hx(c0 - 1) - xf1, hy(c0 - 1));
    g.L0[1] = std::hypot(hx(c0) - xf1, hy(c0));
    g.L0[2] = std::hypot(hx(c0 + 1) - xf1, hy(c0 + 1));
    g.L0[3] = std::hypot(hx(c0 - 1) - xf2, hy(c0 - 1));
    g.L0[4] = std::hypot(hx(c0 + 1) - xf2, hy(c0 + 1));
    return g;
}

// the launch sequence of a (checked) sperm run on stream st
int sperm_forward_impl(swim_ctx* c, int32_t dtype, int64_t n_sys, const swim_sperm_shape& sh,
                       const double* sys_params, const double* swim_params, int32_t steps, double dt,
                       int32_t obs_every, void* head, void* tail, int32_t* status, hipStream_t st)
{
    if (n_sys == 0) return SWIM_OK;
    const SpermShape g = sperm_geometry(sh);
    SpermRun r{};
    r.n_sys = n_sys;
    r.sysp = sys_params;
    r.swp = swim_params;
    r.steps = steps;
    r.dt = dt;
    r.obs_every = obs_every;
    r.n_obs = obs_every > 0 ? steps / obs_every : 0;
    const int n = sh.n_swim * (sh.n_flag + sh.n_head);
    const int tpl = choose_tpl(n);
    // waves per system.  FP32, one-swimmer systems, us per step for 2/4/8
    // waves: 256 systems 11.0/7.0/5.5, 512 11.6/7.8/10.6, 1024 12.0/15.0/20.9,
    // 2000 23.4/29.5/41.4.  The most waves that keep the launch within eight
    // waves per CU.  FP64 is fastest with eight at every size measured.
    int wps = 8;
    if (dtype == SWIM_F32)
        wps = n_sys * 8 <= 8 * (int64_t)c->num_cu ? 8 : n_sys * 4 <= 8 * (int64_t)c->num_cu ? 4 : 2;
    if (c->opt_wps == 2 || c->opt_wps == 4 || c->opt_wps == 8) wps = c->opt_wps;
    void *sysc, *sysc64;
    TRY(sysconst_buffers(c, dtype, n_sys, &sysc, &sysc64));
    if (dtype == SWIM_F32) TRY(ensure(c, B_TAB, (size_t)n_sys * table_bytes()));
    TRY(ensure(c, B_QUEUE, 8 * 4));
    HIPCHK(prepare_sperm(dtype, tpl, wps));
    const int per_cu = sperm_blocks_per_cu(dtype, tpl, wps);
    const int nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(n_sys, (int64_t)per_cu * c->num_cu));
    HIPCHK(launch_sperm_setup(dtype, n_sys, sh.n_swim, sh.eps, sys_params, swim_params, sysc, sysc64, status,
                              c->opt_blob, st));
    if (dtype == SWIM_F32) HIPCHK(launch_table_build(0, n_sys, sysc64, c->buf[B_TAB].p, c->opt_blob, st));
    HIPCHK(launch_fill_i32((int32_t*)c->buf[B_QUEUE].p, 0, 8, st));
    HIPCHK(launch_sperm_forward(dtype, tpl, wps, nblocks, g, r, sysc, dtype == SWIM_F32 ? c->buf[B_TAB].p : nullptr,
                                (int32_t*)c->buf[B_QUEUE].p, head, tail, status, st));
    return SWIM_OK;
}

}  // namespace

extern "C" {

int swim_sperm_forward(swim_ctx* c, int32_t dtype, int64_t n_sys, const swim_sperm_shape* shape,
                       const double* sys_params, const double* swim_params, int32_t steps, double dt,
                       int32_t obs_every, void* head, void* tail, int32_t* status, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n_sys < 0) return fail(SWIM_EINVAL, "n_sys < 0");
    TRY(sperm_check(shape, steps, dt, obs_every));
    if (n_sys == 0) return SWIM_OK;
    if (!sys_params || !swim_params || !head || !tail || !status) return fail(SWIM_EINVAL, "null device pointer");
    return sperm_forward_impl(c, dtype, n_sys, *shape, sys_params, swim_params, steps, dt, obs_every, head, tail,
                              status, pick(c, stream));
}

int swim_sperm_observables(swim_ctx* c, int32_t dtype, int32_t kind, int64_t n_sys, int32_t n_swim, int32_t n_obs,
                           double dt_obs, const void* head, const void* tail, const int32_t* status, double* g,
                           void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (kind != SWIM_OBS_HEAD_VELOCITY && kind != SWIM_OBS_PAIR_DISTANCES) return fail(SWIM_EINVAL, "unknown kind");
    if (n_sys < 0 || n_obs < 1 || n_swim < 1) return fail(SWIM_EINVAL, "bad sizes");
    if (kind == SWIM_OBS_PAIR_DISTANCES && n_swim < 2) return fail(SWIM_EINVAL, "distances need two swimmers");
    if (kind == SWIM_OBS_HEAD_VELOCITY && !(std::isfinite(dt_obs) && dt_obs > 0))
        return fail(SWIM_EINVAL, "dt_obs must be > 0");
    if (n_sys == 0) return SWIM_OK;
    if (!head || !tail || !status || !g) return fail(SWIM_EINVAL, "null device pointer");
    HIPCHK(launch_sperm_observables(dtype, kind, n_sys, n_swim, n_obs, dt_obs, head, tail, status, g,
                                    pick(c, stream)));
    return SWIM_OK;
}

int tmcmc_loglik2(swim_ctx* c, int64_t n, int32_t n_obs, const double* g, const double* data, const double* sigma2,
                  const int32_t* status, double* logl, void* stream)
{
    TRY(check_ctx(c));
    if (n < 0 || n_obs < 1 || (n > 0 && (!g || !data || !sigma2 || !logl)))
        return fail(SWIM_EINVAL, "bad log-likelihood arguments");
    HIPCHK(launch_gauss_loglik2(n, n_obs, g, data, sigma2, status, logl, pick(c, stream)));
    return SWIM_OK;
}

int abc_distance(swim_ctx* c, int32_t dtype, int64_t n, int32_t n_obs, const void* obs, const double* data,
                 const int32_t* status, double* dist, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n < 0 || n_obs < 1) return fail(SWIM_EINVAL, "n must be >= 0 and n_obs >= 1");
    if (n == 0) return SWIM_OK;
    if (!obs || !data || !dist) return fail(SWIM_EINVAL, "null device pointer");
    HIPCHK(launch_abc_distance(dtype, n, n_obs, obs, data, status, dist, pick(c, stream)));
    return SWIM_OK;
}

int abc_select(swim_ctx* c, int64_t n, const double* dist, double q, double* tol, uint8_t* accept, void* stream)
{
    TRY(check_ctx(c));
    if (n < 1) return fail(SWIM_EINVAL, "n must be >= 1");
    if (!(q > 0 && q <= 1)) return fail(SWIM_EINVAL, "quantile must be in (0, 1]");
    if (!dist || !tol) return fail(SWIM_EINVAL, "null device pointer");
    hipStream_t st = pick(c, stream);
    HIPCHK(launch_select_kth(n, dist, q, tol, st));
    if (accept) HIPCHK(launch_accept(n, dist, tol, accept, st));
    return SWIM_OK;
}

int abc_prior_draw(uint64_t seed, int64_t n, int32_t dim, const double* lo, const double* hi, double* theta)
{
    if (n < 0 || dim < 1 || dim > 4 || !lo || !hi || (n > 0 && !theta)) return fail(SWIM_EINVAL, "bad prior-draw arguments");
    for (int d = 0; d < dim; ++d)
        if (!(std::isfinite(lo[d]) && std::isfinite(hi[d]) && hi[d] >= lo[d])) return fail(SWIM_EINVAL, "bad prior box");
    for (int64_t i = 0; i < n; ++i) {
        double u[4];
        uniforms2(seed, 0, (uint64_t)i, 0, u);
        uniforms2(seed, 0, (uint64_t)i, 1, u + 2);
        for (int d = 0; d < dim; ++d) theta[i * dim + d] = lo[d] + (hi[d] - lo[d]) * u[d];
    }
    return SWIM_OK;
}

int abc_pmc_propose(uint64_t seed, int32_t generation, int64_t n, const double* prev_theta, const double* prev_w,
                    int64_t n_prev, const double* lo, const double* hi, double* theta)
{
    if (generation < 1 || n < 0 || n_prev < 1 || !prev_theta || !prev_w || !lo || !hi || (n > 0 && !theta))
        return fail(SWIM_EINVAL, "bad PMC-proposal arguments");
    std::vector<double> cdf(n_prev);
    double acc = 0;
    for (int64_t j = 0; j < n_prev; ++j) {
        if (!(prev_w[j] >= 0 && std::isfinite(prev_w[j]))) return fail(SWIM_EINVAL, "weights must be finite and >= 0");
        acc += prev_w[j];
        cdf[j] = acc;
    }
    if (!(acc > 0)) return fail(SWIM_EINVAL, "weights sum to zero");
    double mu[3], S[9], K[9], L[9];
    wcov3(prev_theta, prev_w, n_prev, mu, S);
    for (int i = 0; i < 9; ++i) K[i] = 2.0 * S[i];
    if (!chol3(K, L)) return fail(SWIM_EINVAL, "perturbation covariance is not positive definite");
    const uint32_t stream = 1u + (uint32_t)generation;
    int bad = 0;
    parallel_for(n, [&](int64_t i) {
        for (int a = 0; a < 10000; ++a) {
            double u01[2], u23[2], u45[2];
            uniforms2(seed, stream, (uint64_t)i, 3u * a, u01);
            uniforms2(seed, stream, (uint64_t)i, 3u * a + 1, u23);
            uniforms2(seed, stream, (uint64_t)i, 3u * a + 2, u45);
            int64_t j = std::upper_bound(cdf.begin(), cdf.end(), u01[0] * cdf.back()) - cdf.begin();
            if (j >= n_prev) j = n_prev - 1;
            double z[3], zz;
            box_muller(u01[1], u23[0], &z[0], &z[1]);
            box_muller(u23[1], u45[0], &z[2], &zz);
            double cand[3];
            bool in = true;
            for (int d = 0; d < 3; ++d) {
                double v = prev_theta[3 * j + d];
                for (int e = 0; e <= d; ++e) v += L[3 * d + e] * z[e];
                cand[d] = v;
                in = in && v >= lo[d] && v <= hi[d];
            }
            if (in) {
                for (int d = 0; d < 3; ++d) theta[3 * i + d] = cand[d];
                return;
            }
        }
        bad = 1;
    });
    if (bad) return fail(SWIM_EINVAL, "PMC proposal could not be placed inside the prior box");
    return SWIM_OK;
}

int abc_pmc_weights(int64_t n, const double* theta, const uint8_t* accept, const double* prev_theta,
                    const double* prev_w, int64_t n_prev, double* w)
{
    if (n < 0 || n_prev < 1 || !theta || !accept || !prev_theta || !prev_w || !w) return fail(SWIM_EINVAL, "bad PMC-weight arguments");
    double pws = 0;
    for (int64_t j = 0; j < n_prev; ++j) pws += prev_w[j];
    if (!(pws > 0)) return fail(SWIM_EINVAL, "weights sum to zero");
    double mu[3], S[9], K[9], L[9];
    wcov3(prev_theta, prev_w, n_prev, mu, S);
    for (int i = 0; i < 9; ++i) K[i] = 2.0 * S[i];
    if (!chol3(K, L)) return fail(SWIM_EINVAL, "perturbation covariance is not positive definite");
    parallel_for(n, [&](int64_t i) {
        if (!accept[i]) {
            w[i] = 0;
            return;
        }
        double dens = 0;
        for (int64_t j = 0; j < n_prev; ++j) {
            double d[3], y[3];
            for (int e = 0; e < 3; ++e) d[e] = theta[3 * i + e] - prev_theta[3 * j + e];
            // solve L y = d;  quadratic form = |y|^2
            for (int a = 0; a < 3; ++a) {
                double s = d[a];
                for (int e = 0; e < a; ++e) s -= L[3 * a + e] * y[e];
                y[a] = s / L[3 * a + a];
            }
            dens += (prev_w[j] / pws) * std::exp(-0.5 * (y[0] * y[0] + y[1] * y[1] + y[2] * y[2]));
        }
        w[i] = 1.0 / dens;
    });
    double tot = 0;
    for (int64_t i = 0; i < n; ++i) tot += w[i];
    if (!(tot > 0) || !std::isfinite(tot)) return fail(SWIM_EINVAL, "no accepted proposal has a finite weight");
    for (int64_t i = 0; i < n; ++i) w[i] /= tot;
    return SWIM_OK;
}

int abc_step(swim_ctx* c, const abc_model* m, const double* data, int32_t n_obs, int64_t n, const int32_t* N,
             uint64_t seed, int32_t generation, const double* prev_theta, const double* prev_w, int64_t n_prev, double q,
             double* theta_out, double* dist_out, uint8_t* accept_out, double* w_out, double* tol_out,
             int32_t* steps_out)
{
    TRY(check_ctx(c));
    if (!m || !data || !N || !theta_out || !dist_out || !accept_out || !w_out || !tol_out) return fail(SWIM_EINVAL, "null argument");
    TRY(check_dtype(m->dtype));
    if (n < 1) return fail(SWIM_EINVAL, "n must be >= 1");
    if (m->obs_every < 1 || n_obs != m->steps / m->obs_every) return fail(SWIM_EINVAL, "n_obs must equal steps/obs_every");
    TRY(check_run(n, N, nullptr, m->steps, m->dt, m->obs_every, m->eps_over_ds));
    if (!(q > 0 && q <= 1)) return fail(SWIM_EINVAL, "quantile must be in (0, 1]");
    // proposals
    if (generation == 0) {
        TRY(abc_prior_draw(seed, n, 3, m->lo, m->hi, theta_out));
    } else {
        TRY(abc_pmc_propose(seed, generation, n, prev_theta, prev_w, n_prev, m->lo, m->hi, theta_out));
    }
    std::vector<double> rows((size_t)n * SWIM_NPARAM);
    for (int64_t i = 0; i < n; ++i) {
        double* P = &rows[(size_t)i * SWIM_NPARAM];
        P[0] = theta_out[3 * i];
        P[1] = theta_out[3 * i + 1];
        P[2] = theta_out[3 * i + 2];
        P[3] = m->b;
        P[4] = m->omega;
        P[5] = m->k;
        P[6] = 0.0;
        P[7] = 0.0;
        P[8] = 0.0;
    }
    hipStream_t st = c->stream;
    const size_t es = m->dtype == SWIM_F32 ? 4 : 8;
    TRY(ensure(c, B_OBS, (size_t)n * n_obs * 2 * es));
    TRY(ensure(c, B_SPEED, (size_t)n * es));
    TRY(ensure(c, B_STATUS, (size_t)n * 4));
    TRY(ensure(c, B_DIST, (size_t)n * 8));
    TRY(ensure(c, B_TOL, 8));
    TRY(ensure(c, B_ACC, (size_t)n));
    TRY(begin_uploads(c, rows.size() * 8 + (size_t)n_obs * 16));
    TRY(stage(c, rows.data(), rows.size() * 8, B_PARAMS, st));
    TRY(stage(c, data, (size_t)n_obs * 16, B_DATA, st));
    TRY(end_uploads(c, st));
    Run r;
    r.steps = m->steps;
    r.dt = m->dt;
    r.obs_every = m->obs_every;
    r.n_obs = n_obs;
    r.eps_over_ds = m->eps_over_ds;
    if (steps_out) TRY(ensure(c, B_DONE, (size_t)n * 4));
    int32_t* done_dev = steps_out ? (int32_t*)c->buf[B_DONE].p : nullptr;
    const int save_graph = c->opt_graph;
    if (!m->use_graph) c->opt_graph = 0;
    const int frc = forward_impl(c, m->dtype, n, N, nullptr, (const double*)c->buf[B_PARAMS].p, r, c->buf[B_OBS].p,
                                 c->buf[B_SPEED].p, (int32_t*)c->buf[B_STATUS].p, done_dev, st);
    c->opt_graph = save_graph;
    TRY(frc);
    HIPCHK(launch_abc_distance(m->dtype, n, n_obs, c->buf[B_OBS].p, (const double*)c->buf[B_DATA].p,
                               (const int32_t*)c->buf[B_STATUS].p, (double*)c->buf[B_DIST].p, st));
    HIPCHK(launch_select_kth(n, (const double*)c->buf[B_DIST].p, q, (double*)c->buf[B_TOL].p, st));
    HIPCHK(launch_accept(n, (const double*)c->buf[B_DIST].p, (const double*)c->buf[B_TOL].p, (uint8_t*)c->buf[B_ACC].p, st));
    HIPCHK(hipMemcpyAsync(dist_out, c->buf[B_DIST].p, (size_t)n * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(accept_out, c->buf[B_ACC].p, (size_t)n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(tol_out, c->buf[B_TOL].p, 8, hipMemcpyDeviceToHost, st));
    if (steps_out) HIPCHK(hipMemcpyAsync(steps_out, done_dev, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (generation == 0) {
        int64_t na = 0;
        for (int64_t i = 0; i < n; ++i) na += accept_out[i] ? 1 : 0;
        for (int64_t i = 0; i < n; ++i) w_out[i] = (accept_out[i] && na) ? 1.0 / (double)na : 0.0;
    } else {
        TRY(abc_pmc_weights(n, theta_out, accept_out, prev_theta, prev_w, n_prev, w_out));
    }
    return SWIM_OK;
}

int swim_forward_plan(int32_t dtype, int64_t n_sys, const int32_t* N, const int32_t* n_swim, double eps_over_ds,
                      int32_t* tpl)
{
    TRY(check_dtype(dtype));
    if (n_sys < 0 || (n_sys > 0 && (!N || !tpl))) return fail(SWIM_EINVAL, "bad swim_forward_plan arguments");
    if (!(eps_over_ds > 0)) return fail(SWIM_EINVAL, "eps_over_ds must be > 0");
    bool present[9] = {}, big = false;
    for (int64_t s = 0; s < n_sys; ++s) {
        const int nsw = n_swim ? n_swim[s] : 1;
        if (N[s] < 3 || N[s] > 4096 || nsw < 1 || (int64_t)N[s] * nsw > 4096)
            return fail(SWIM_EINVAL, "system %lld: N = %d with %d filaments is outside the limits", (long long)s, N[s], nsw);
        const int t = forward_tpl(dtype, N[s], N[s] * nsw, eps_over_ds);
        if (t > 0) present[t] = true;
        else big = true;
    }
    int launch[9];
    merge_buckets(present, big, 1 + swim_ctx::N_AUX, launch);
    for (int64_t s = 0; s < n_sys; ++s) {
        const int nsw = n_swim ? n_swim[s] : 1;
        const int t = forward_tpl(dtype, N[s], N[s] * nsw, eps_over_ds);
        tpl[s] = t > 0 ? launch[t] : -1;
    }
    return SWIM_OK;
}

int swim_kernel_eval_host(int32_t dtype, double alpha, double eps, int32_t blob, int64_t n, const double* t,
                          double* h1t, double* h2, double* h1c)
{
    TRY(check_dtype(dtype));
    if (blob != SWIM_BLOB_READING && blob != SWIM_BLOB_PAPER) return fail(SWIM_EINVAL, "blob must be 0 or 1");
    if (!(std::isfinite(alpha) && alpha >= 0 && std::isfinite(eps) && eps > 0 && alpha * eps <= 1.0))
        return fail(SWIM_EINVAL, "alpha/eps outside the domain");
    if (n < 0 || (n > 0 && (!t || !h1t || !h2)) || !h1c) return fail(SWIM_EINVAL, "bad arguments");
    if (dtype == SWIM_F32) {
        // the device's FP32 path: the per-system table, direct evaluation
        // beyond its last octave
        SysConst<float> C;
        sysconst_compute<float>(alpha, eps, &C, blob);
        SysConst<double> C64;
        sysconst_compute<double>(alpha, eps, &C64, blob);
        std::vector<TabE> tab(TAB_N + 1);
        if (C64.paper == 2.0) {
            // the paper's blob at alpha > 0: the nodes from the sweep
            std::vector<double> fh(PB_NODES), fg(PB_NODES);
            pb_table_nodes_host(C64, fh.data(), fg.data());
            for (int i = 0; i < TAB_N; ++i) {
                const double h4[4] = {fh[3 * i], fh[3 * i + 1], fh[3 * i + 2], fh[3 * i + 3]};
                const double g4[4] = {fg[3 * i], fg[3 * i + 1], fg[3 * i + 2], fg[3 * i + 3]};
                tab_assemble(C64, h4, g4, tab[i], nullptr);
            }
            tab_interval(C64, TAB_N, tab[TAB_N], nullptr);
        } else {
            for (int i = 0; i <= TAB_N; ++i) tab_interval(C64, i, tab[i], nullptr);
        }
        for (int64_t i = 0; i < n; ++i) {
            float a, b;
            const float tf = (float)t[i];
            const uint32_t bits = tab_bits(tf, C.ts);
            const uint32_t k = bits >> TAB_SHIFT;
            if (k < TAB_END) {
                tab_eval(tab[k - TAB_BIAS], tab_u(bits), a, b);
                b *= C.ts;  // the table holds H2 / sigma
            } else {
                kernel_eval<float>(C, tf, a, b);
            }
            h1t[i] = a;
            h2[i] = b;
        }
        *h1c = C.h1c;
    } else {
        SysConst<double> C;
        sysconst_compute<double>(alpha, eps, &C, blob);
        for (int64_t i = 0; i < n; ++i) {
            double a, b;
            kernel_eval<double>(C, t[i], a, b);
            h1t[i] = a;
            h2[i] = b;
        }
        *h1c = C.h1c;
    }
    return SWIM_OK;
}

// ==========================================================================
// surrogate
// ==========================================================================
int surrogate_forward(swim_ctx* c, int64_t n, const float* X, const float* params, float* Y, void* stream)
{
    TRY(check_ctx(c));
    if (n < 0 || (n > 0 && (!X || !params || !Y))) return fail(SWIM_EINVAL, "bad surrogate_forward arguments");
    hipStream_t st = pick(c, stream);
    if (n == 0) return SWIM_OK;
    TRY(ensure(c, B_W16, (size_t)mlp_w16_count() * 2));
    HIPCHK(launch_pack_w16(params, (uint16_t*)c->buf[B_W16].p, st));
    HIPCHK(launch_mlp_fused(0, n, X, (const uint16_t*)c->buf[B_W16].p, params, Y, nullptr, nullptr, nullptr, 0, 0.f,
                            nullptr, nullptr, st));
    return SWIM_OK;
}

}  // extern "C"

namespace {

// surrogate distance of n standardized inputs (fused MLP kernel: the
// activations never leave LDS), then the compaction of the kept rows
int prescreen_impl(swim_ctx* c, int64_t n, const float* X, const float* params, const float* out_mu,
                   const float* out_sd, const float* obs_sum, int32_t n_sum, float tol, float* dist, uint8_t* keep,
                   int64_t* idx, int64_t* n_keep, hipStream_t st)
{
    TRY(ensure(c, B_W16, (size_t)mlp_w16_count() * 2));
    HIPCHK(launch_pack_w16(params, (uint16_t*)c->buf[B_W16].p, st));
    HIPCHK(launch_mlp_fused(1, n, X, (const uint16_t*)c->buf[B_W16].p, params, nullptr, out_mu, out_sd, obs_sum, n_sum,
                            tol, dist, keep, st));
    TRY(ensure(c, B_MLP_CNT, (size_t)((n + 255) / 256) * 4));
    HIPCHK(launch_compact(n, keep, (int32_t*)c->buf[B_MLP_CNT].p, idx, n_keep, st));
    return SWIM_OK;
}
}  // namespace

extern "C" {

int surrogate_grad(swim_ctx* c, int64_t n, const float* X, const float* T, const float* params, float* grads,
                   float* loss, void* stream)
{
    TRY(check_ctx(c));
    if (n < 1 || n > (1 << 20) || !X || !T || !params || !grads) return fail(SWIM_EINVAL, "bad surrogate_grad arguments");
    hipStream_t st = pick(c, stream);
    MlpAct a;
    TRY(mlp_act(c, n, &a));
    TRY(mlp_forward(X, params, n, a, a.Y, st, T));
    TRY(mlp_backward(X, params, n, a, grads, loss, st));
    return SWIM_OK;
}

int surrogate_train(swim_ctx* c, int64_t n, const float* X, const float* T, const int32_t* perm, int32_t epochs,
                    int32_t batch, float lr, float* params, float* adam_m, float* adam_v, float* loss_out, void* stream)
{
    TRY(check_ctx(c));
    if (n < 1 || epochs < 1 || batch < 1 || batch > n || batch > (1 << 16) || !(lr > 0) || !X || !T || !perm || !params ||
        !adam_m || !adam_v)
        return fail(SWIM_EINVAL, "bad surrogate_train arguments");
    hipStream_t st = pick(c, stream);
    MlpAct a;
    TRY(mlp_act(c, batch, &a));
    TRY(ensure(c, B_MLP_GRAD, (size_t)MLP_NPARAM * 4));
    TRY(ensure(c, B_MLP_BATCH, (size_t)batch * (MLP_W[0] + MLP_W[MLP_L]) * 4));
    float* G = (float*)c->buf[B_MLP_GRAD].p;
    float* Xb = (float*)c->buf[B_MLP_BATCH].p;
    float* Tb = Xb + (size_t)batch * MLP_W[0];
    const int64_t spe = n / batch;
    const double b1 = 0.9, b2 = 0.999;
    int64_t t = 0;
    for (int e = 0; e < epochs; ++e) {
        for (int64_t s = 0; s < spe; ++s) {
            ++t;
            HIPCHK(launch_gather_rows(batch, perm + (int64_t)e * n + s * batch, n, X, MLP_W[0], T, MLP_W[MLP_L], Xb, Tb,
                                      st));
            TRY(mlp_forward(Xb, params, batch, a, a.Y, st, Tb));
            TRY(mlp_backward(Xb, params, batch, a, G, loss_out ? loss_out + e * spe + s : nullptr, st));
            HIPCHK(launch_adam(MLP_NPARAM, params, G, adam_m, adam_v, lr, (float)b1, (float)b2,
                               (float)(1.0 - std::pow(b1, (double)t)), (float)(1.0 - std::pow(b2, (double)t)), 1e-8f, st));
        }
    }
    return SWIM_OK;
}

int surrogate_prescreen(swim_ctx* c, int64_t n, const float* X, const float* params, const float* out_mu,
                        const float* out_sd, const float* obs_sum, int32_t n_sum, float tol, float* dist, uint8_t* keep,
                        int64_t* idx, int64_t* n_keep, void* stream)
{
    TRY(check_ctx(c));
    if (n < 1 || n_sum < 1 || n_sum > MLP_W[MLP_L] || !(tol >= 0) || !X || !params || !out_mu || !out_sd || !obs_sum ||
        !keep || !idx || !n_keep)
        return fail(SWIM_EINVAL, "bad surrogate_prescreen arguments");
    return prescreen_impl(c, n, X, params, out_mu, out_sd, obs_sum, n_sum, tol, dist, keep, idx, n_keep,
                          pick(c, stream));
}

int surrogate_features(swim_ctx* c, int64_t n, const double* theta, double b, double omega, const float* mu,
                       const float* sd, float* X, void* stream)
{
    TRY(check_ctx(c));
    if (n < 0 || (n > 0 && (!theta || !X)) || ((mu == nullptr) != (sd == nullptr)))
        return fail(SWIM_EINVAL, "bad surrogate_features arguments");
    HIPCHK(launch_features(n, theta, b, omega, mu, sd, X, pick(c, stream)));
    return SWIM_OK;
}

int surrogate_targets(swim_ctx* c, int32_t dtype, int64_t n, int32_t n_obs, const void* obs, const void* speed,
                      double x0, double y0, const int32_t* sum_idx, int32_t n_sum, float* T, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n < 0 || n_obs < 1 || n_sum < 1 || n_sum > 64 || !sum_idx || (n > 0 && (!obs || !speed || !T)))
        return fail(SWIM_EINVAL, "bad surrogate_targets arguments");
    for (int j = 0; j < n_sum; ++j)
        if (sum_idx[j] < 0 || sum_idx[j] >= n_obs) return fail(SWIM_EINVAL, "summary index %d out of range", sum_idx[j]);
    hipStream_t st = pick(c, stream);
    TRY(begin_uploads(c, (size_t)n_sum * 4));
    TRY(stage(c, sum_idx, (size_t)n_sum * 4, B_MLP_IDX, st));
    TRY(end_uploads(c, st));
    HIPCHK(launch_targets(dtype, n, n_obs, obs, speed, x0, y0, (const int32_t*)c->buf[B_MLP_IDX].p, n_sum, T, st));
    return SWIM_OK;
}

int surrogate_colstats(swim_ctx* c, int64_t n, int32_t cols, const float* A, float* mu, float* sd, void* stream)
{
    TRY(check_ctx(c));
    if (n < 1 || cols < 1 || !A || !mu || !sd) return fail(SWIM_EINVAL, "bad surrogate_colstats arguments");
    HIPCHK(launch_colstats(n, cols, A, mu, sd, pick(c, stream)));
    return SWIM_OK;
}

int surrogate_standardize(swim_ctx* c, int64_t n, int32_t cols, float* A, const float* mu, const float* sd,
                          void* stream)
{
    TRY(check_ctx(c));
    if (n < 0 || cols < 1 || (n > 0 && (!A || !mu || !sd))) return fail(SWIM_EINVAL, "bad surrogate_standardize arguments");
    HIPCHK(launch_standardize(n, cols, A, mu, sd, pick(c, stream)));
    return SWIM_OK;
}

int abc_prior_draw_device(swim_ctx* c, uint64_t seed, int64_t n, const double* lo, const double* hi, double* theta,
                          void* stream)
{
    TRY(check_ctx(c));
    if (n < 0 || !lo || !hi || (n > 0 && !theta)) return fail(SWIM_EINVAL, "bad prior-draw arguments");
    for (int d = 0; d < 3; ++d)
        if (!(std::isfinite(lo[d]) && std::isfinite(hi[d]) && hi[d] >= lo[d])) return fail(SWIM_EINVAL, "bad prior box");
    HIPCHK(launch_prior_draw(seed, n, lo, hi, theta, pick(c, stream)));
    return SWIM_OK;
}

int swim_param_rows(swim_ctx* c, int64_t cap, const int64_t* n_dev, const int64_t* idx, int64_t n_theta,
                    const double* theta, double b, double omega, double k, double* rows, void* stream)
{
    TRY(check_ctx(c));
    if (cap < 0 || n_theta < 0 || (cap > 0 && (!theta || !rows))) return fail(SWIM_EINVAL, "bad swim_param_rows arguments");
    if (!idx && cap > n_theta) return fail(SWIM_EINVAL, "cap exceeds n_theta");
    HIPCHK(launch_param_rows(cap, n_dev, idx, n_theta, theta, b, omega, k, rows, pick(c, stream)));
    return SWIM_OK;
}

int swim_select(swim_ctx* c, int64_t n, const int32_t* values, int32_t want, uint8_t* keep, int64_t* idx,
                int64_t* n_keep, void* stream)
{
    TRY(check_ctx(c));
    if (n < 1 || !keep || !idx || !n_keep) return fail(SWIM_EINVAL, "bad swim_select arguments");
    hipStream_t st = pick(c, stream);
    if (values) HIPCHK(launch_flag_eq(n, values, want, keep, st));
    TRY(ensure(c, B_MLP_CNT, (size_t)((n + 255) / 256) * 4));
    HIPCHK(launch_compact(n, keep, (int32_t*)c->buf[B_MLP_CNT].p, idx, n_keep, st));
    return SWIM_OK;
}

int swim_gather_rows(swim_ctx* c, int64_t cap, const int64_t* n_dev, const int64_t* idx, int64_t n_src,
                     const float* src, int32_t cols, float* dst, void* stream)
{
    TRY(check_ctx(c));
    if (cap < 0 || cols < 1 || n_src < 0 || (cap > 0 && (!n_dev || !idx || !src || !dst)))
        return fail(SWIM_EINVAL, "bad swim_gather_rows arguments");
    HIPCHK(launch_gather_f32(cap, n_dev, idx, n_src, src, cols, dst, pick(c, stream)));
    return SWIM_OK;
}

int surrogate_dataset(swim_ctx* c, const abc_model* m, int32_t N, int64_t n_runs, uint64_t seed, const int32_t* sum_idx,
                      int32_t n_sum, double max_disp, int64_t cap, float* X, float* T, float* in_mu, float* in_sd,
                      float* out_mu, float* out_sd, int64_t* n_out, void* stream)
{
    TRY(check_ctx(c));
    if (!m || !sum_idx || !n_out || !X || !T || !in_mu || !in_sd || !out_mu || !out_sd)
        return fail(SWIM_EINVAL, "null argument");
    TRY(check_dtype(m->dtype));
    if (n_runs < 1 || cap < 1) return fail(SWIM_EINVAL, "n_runs and cap must be >= 1");
    if (!(max_disp > 0)) return fail(SWIM_EINVAL, "max_disp must be > 0");
    if (2 * n_sum + 1 != MLP_W[MLP_L]) return fail(SWIM_EINVAL, "n_sum must be %d", (MLP_W[MLP_L] - 1) / 2);
    if (m->obs_every < 1) return fail(SWIM_EINVAL, "obs_every must be >= 1");
    const int32_t n_obs = m->steps / m->obs_every;
    for (int j = 0; j < n_sum; ++j)
        if (sum_idx[j] < 0 || sum_idx[j] >= n_obs) return fail(SWIM_EINVAL, "summary index %d out of range", sum_idx[j]);
    for (int d = 0; d < 3; ++d)
        if (!(std::isfinite(m->lo[d]) && std::isfinite(m->hi[d]) && m->hi[d] >= m->lo[d] && m->lo[d] >= 0))
            return fail(SWIM_EINVAL, "bad prior box");
    if (!(m->lo[1] > 0 && m->lo[2] > 0)) return fail(SWIM_EINVAL, "the prior of S_b and S_s must be positive (log inputs)");
    std::vector<int32_t> Nv((size_t)n_runs, N);
    TRY(check_run(n_runs, Nv.data(), nullptr, m->steps, m->dt, m->obs_every, m->eps_over_ds));
    hipStream_t st = pick(c, stream);
    const size_t es = m->dtype == SWIM_F32 ? 4 : 8;
    const int nx = MLP_W[0], nt = MLP_W[MLP_L];
    TRY(ensure(c, B_PS_THETA, (size_t)n_runs * 24));
    TRY(ensure(c, B_PARAMS, (size_t)n_runs * SWIM_NPARAM * 8));
    TRY(ensure(c, B_OBS, (size_t)n_runs * n_obs * 2 * es));
    TRY(ensure(c, B_SPEED, (size_t)n_runs * es));
    TRY(ensure(c, B_STATUS, (size_t)n_runs * 4));
    TRY(ensure(c, B_PS_KEEP, (size_t)n_runs));
    TRY(ensure(c, B_PS_IDX, (size_t)n_runs * 8));
    TRY(ensure(c, B_PS_NK, 8));
    TRY(ensure(c, B_PS_X, (size_t)n_runs * nx * 4));
    TRY(ensure(c, B_DS_T, (size_t)n_runs * nt * 4));
    double* theta = (double*)c->buf[B_PS_THETA].p;
    double* rows = (double*)c->buf[B_PARAMS].p;
    HIPCHK(launch_prior_draw(seed, n_runs, m->lo, m->hi, theta, st));
    HIPCHK(launch_param_rows(n_runs, nullptr, nullptr, n_runs, theta, m->b, m->omega, m->k, rows, st));
    Run r;
    r.steps = m->steps;
    r.dt = m->dt;
    r.obs_every = m->obs_every;
    r.n_obs = n_obs;
    r.eps_over_ds = m->eps_over_ds;
    TRY(forward_impl(c, m->dtype, n_runs, Nv.data(), nullptr, rows, r, c->buf[B_OBS].p, c->buf[B_SPEED].p,
                     (int32_t*)c->buf[B_STATUS].p, nullptr, st));
    float* Xall = (float*)c->buf[B_PS_X].p;
    float* Tall = (float*)c->buf[B_DS_T].p;
    HIPCHK(launch_features(n_runs, theta, m->b, m->omega, nullptr, nullptr, Xall, st));
    TRY(begin_uploads(c, (size_t)n_sum * 4));
    TRY(stage(c, sum_idx, (size_t)n_sum * 4, B_MLP_IDX, st));
    TRY(end_uploads(c, st));
    // the head starts at (L, 0) = (1, 0): parameter rows carry a zero offset
    HIPCHK(launch_targets(m->dtype, n_runs, n_obs, c->buf[B_OBS].p, c->buf[B_SPEED].p, 1.0, 0.0,
                          (const int32_t*)c->buf[B_MLP_IDX].p, n_sum, Tall, st));
    uint8_t* keep = (uint8_t*)c->buf[B_PS_KEEP].p;
    int64_t* idx = (int64_t*)c->buf[B_PS_IDX].p;
    int64_t* nk = (int64_t*)c->buf[B_PS_NK].p;
    HIPCHK(launch_flag_eq(n_runs, (const int32_t*)c->buf[B_STATUS].p, SWIM_ST_OK, keep, st));
    HIPCHK(launch_flag_bounded(n_runs, Tall, nt, 2 * n_sum, (float)max_disp, keep, st));
    TRY(ensure(c, B_MLP_CNT, (size_t)((n_runs + 255) / 256) * 4));
    HIPCHK(launch_compact(n_runs, keep, (int32_t*)c->buf[B_MLP_CNT].p, idx, nk, st));
    int64_t n_keep = 0;
    HIPCHK(hipMemcpyAsync(&n_keep, nk, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t n = std::min(n_keep, cap);
    *n_out = n;
    if (n == 0) return SWIM_OK;
    HIPCHK(launch_gather_f32(n, nk, idx, n_runs, Xall, nx, X, st));
    HIPCHK(launch_gather_f32(n, nk, idx, n_runs, Tall, nt, T, st));
    HIPCHK(launch_colstats(n, nx, X, in_mu, in_sd, st));
    HIPCHK(launch_standardize(n, nx, X, in_mu, in_sd, st));
    HIPCHK(launch_colstats(n, nt, T, out_mu, out_sd, st));
    HIPCHK(launch_standardize(n, nt, T, out_mu, out_sd, st));
    return SWIM_OK;
}

int abc_prescreened(swim_ctx* c, const abc_model* m, int32_t N, const float* params, const float* in_mu,
                    const float* in_sd, const float* out_mu, const float* out_sd, const int32_t* sum_idx,
                    int32_t n_sum, const double* data, int32_t n_obs, double tol, double factor, int64_t n_prop,
                    uint64_t seed, int64_t cap, double* theta_out, double* dist_out, uint8_t* accept_out,
                    int64_t* n_surv, float* ms_out)
{
    TRY(check_ctx(c));
    if (!m || !params || !in_mu || !in_sd || !out_mu || !out_sd || !sum_idx || !data || !n_surv ||
        (cap > 0 && (!theta_out || !dist_out || !accept_out)))
        return fail(SWIM_EINVAL, "null argument");
    TRY(check_dtype(m->dtype));
    if (n_prop < 1 || cap < 0) return fail(SWIM_EINVAL, "n_prop must be >= 1 and cap >= 0");
    if (!(tol >= 0) || !(factor > 0) || !std::isfinite(tol * factor)) return fail(SWIM_EINVAL, "bad tolerance");
    if (2 * n_sum + 1 != MLP_W[MLP_L]) return fail(SWIM_EINVAL, "n_sum must be %d", (MLP_W[MLP_L] - 1) / 2);
    if (m->obs_every < 1 || n_obs != m->steps / m->obs_every) return fail(SWIM_EINVAL, "n_obs must equal steps/obs_every");
    for (int j = 0; j < n_sum; ++j)
        if (sum_idx[j] < 0 || sum_idx[j] >= n_obs) return fail(SWIM_EINVAL, "summary index %d out of range", sum_idx[j]);
    for (int d = 0; d < 3; ++d)
        if (!(std::isfinite(m->lo[d]) && std::isfinite(m->hi[d]) && m->hi[d] >= m->lo[d] && m->lo[d] >= 0))
            return fail(SWIM_EINVAL, "bad prior box");
    if (!(m->lo[1] > 0 && m->lo[2] > 0)) return fail(SWIM_EINVAL, "the prior of S_b and S_s must be positive (log inputs)");
    {
        const int32_t N1 = N;
        TRY(check_run(1, &N1, nullptr, m->steps, m->dt, m->obs_every, m->eps_over_ds));
    }
    hipStream_t st = c->stream;
    const size_t es = m->dtype == SWIM_F32 ? 4 : 8;
    const int nx = MLP_W[0];
    // observed summaries: head displacement from its start (1, 0)
    std::vector<float> osum(2 * n_sum);
    for (int j = 0; j < n_sum; ++j) {
        osum[2 * j] = (float)(data[2 * sum_idx[j]] - 1.0);
        osum[2 * j + 1] = (float)data[2 * sum_idx[j] + 1];
    }
    TRY(ensure(c, B_PS_THETA, (size_t)n_prop * 24));
    TRY(ensure(c, B_PS_X, (size_t)n_prop * nx * 4));
    TRY(ensure(c, B_PS_KEEP, (size_t)n_prop));
    TRY(ensure(c, B_PS_IDX, (size_t)n_prop * 8));
    TRY(ensure(c, B_PS_NK, 8));
    TRY(begin_uploads(c, osum.size() * 4 + (size_t)n_obs * 16 + 8));
    TRY(stage(c, osum.data(), osum.size() * 4, B_PS_SUM, st));
    TRY(stage(c, data, (size_t)n_obs * 16, B_DATA, st));
    TRY(stage(c, &tol, 8, B_TOL, st));
    TRY(end_uploads(c, st));
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard()
        {
            for (int i = 0; i < 3; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};
    if (ms_out)
        for (int i = 0; i < 3; ++i) HIPCHK(hipEventCreate(&ev[i]));
    if (ms_out) HIPCHK(hipEventRecord(ev[0], st));
    double* theta = (double*)c->buf[B_PS_THETA].p;
    float* X = (float*)c->buf[B_PS_X].p;
    int64_t* idx = (int64_t*)c->buf[B_PS_IDX].p;
    int64_t* nk = (int64_t*)c->buf[B_PS_NK].p;
    HIPCHK(launch_prior_draw(seed, n_prop, m->lo, m->hi, theta, st));
    HIPCHK(launch_features(n_prop, theta, m->b, m->omega, in_mu, in_sd, X, st));
    TRY(prescreen_impl(c, n_prop, X, params, out_mu, out_sd, (const float*)c->buf[B_PS_SUM].p, 2 * n_sum,
                       (float)(factor * tol), nullptr, (uint8_t*)c->buf[B_PS_KEEP].p, idx, nk, st));
    if (ms_out) HIPCHK(hipEventRecord(ev[1], st));
    int64_t n_keep = 0;
    HIPCHK(hipMemcpyAsync(&n_keep, nk, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *n_surv = n_keep;
    const int64_t n = std::min(n_keep, cap);
    if (n > 0) {
        TRY(ensure(c, B_PARAMS, (size_t)n * SWIM_NPARAM * 8));
        TRY(ensure(c, B_OBS, (size_t)n * n_obs * 2 * es));
        TRY(ensure(c, B_SPEED, (size_t)n * es));
        TRY(ensure(c, B_STATUS, (size_t)n * 4));
        TRY(ensure(c, B_DIST, (size_t)n * 8));
        TRY(ensure(c, B_ACC, (size_t)n));
        double* rows = (double*)c->buf[B_PARAMS].p;
        HIPCHK(launch_param_rows(n, nk, idx, n_prop, theta, m->b, m->omega, m->k, rows, st));
        std::vector<int32_t> Nv((size_t)n, N);
        Run r;
        r.steps = m->steps;
        r.dt = m->dt;
        r.obs_every = m->obs_every;
        r.n_obs = n_obs;
        r.eps_over_ds = m->eps_over_ds;
        // the tolerance is known: a survivor stops as soon as its running
        // sum of squared head deviations exceeds 2 n_obs tol^2 (a hair
        // above, so that rounding never rejects a run the distance accepts)
        if (c->opt_early_stop) {
            r.stop_data = (const double*)c->buf[B_DATA].p;
            r.stop_ssq = 2.0 * n_obs * tol * tol * (1.0 + 1e-6);
        }
        TRY(forward_impl(c, m->dtype, n, Nv.data(), nullptr, rows, r, c->buf[B_OBS].p, c->buf[B_SPEED].p,
                         (int32_t*)c->buf[B_STATUS].p, nullptr, st));
        HIPCHK(launch_abc_distance(m->dtype, n, n_obs, c->buf[B_OBS].p, (const double*)c->buf[B_DATA].p,
                                   (const int32_t*)c->buf[B_STATUS].p, (double*)c->buf[B_DIST].p, st));
        HIPCHK(launch_accept(n, (const double*)c->buf[B_DIST].p, (const double*)c->buf[B_TOL].p,
                             (uint8_t*)c->buf[B_ACC].p, st));
    }
    if (ms_out) HIPCHK(hipEventRecord(ev[2], st));
    std::vector<double> hrows((size_t)n * SWIM_NPARAM);
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(hrows.data(), c->buf[B_PARAMS].p, hrows.size() * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(dist_out, c->buf[B_DIST].p, (size_t)n * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(accept_out, c->buf[B_ACC].p, (size_t)n, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) theta_out[3 * i + d] = hrows[(size_t)i * SWIM_NPARAM + d];
    if (ms_out) {
        HIPCHK(hipEventElapsedTime(&ms_out[0], ev[0], ev[1]));
        HIPCHK(hipEventElapsedTime(&ms_out[1], ev[1], ev[2]));
    }
    return SWIM_OK;
}


// ==========================================================================
// autotuner
// ==========================================================================
int swim_autotune(swim_ctx* c, int32_t dtype, int64_t n_sys, const int32_t* N, const int32_t* n_swim,
                  const double* params, int32_t probe_steps, double dt, double eps_over_ds, int32_t* chosen)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n_sys < 1 || !N || !params || !chosen) return fail(SWIM_EINVAL, "bad swim_autotune arguments");
    if (probe_steps < 1) return fail(SWIM_EINVAL, "probe_steps must be >= 1");
    TRY(check_run(n_sys, N, n_swim, probe_steps, dt, probe_steps, eps_over_ds));
    hipStream_t st = c->stream;
    int64_t nfil = 0;
    bool present[9] = {}, has_tpl[9] = {};
    bool has_big = false;
    for (int64_t s = 0; s < n_sys; ++s) {
        const int nsw = n_swim ? n_swim[s] : 1;
        nfil += nsw;
        const int tpl = forward_tpl(dtype, N[s], N[s] * nsw, eps_over_ds);
        if (tpl > 0) present[tpl] = true;
        else has_big = true;
    }
    // the buckets the forward calls launch (merge_buckets)
    int launch_tpl[9];
    merge_buckets(present, has_big, 1 + swim_ctx::N_AUX, launch_tpl);
    for (int t = 1; t <= 8; ++t)
        if (launch_tpl[t] > 0) has_tpl[launch_tpl[t]] = true;
    const size_t es = dtype == SWIM_F32 ? 4 : 8;
    TRY(ensure(c, B_OBS, (size_t)nfil * 2 * es));
    TRY(ensure(c, B_SPEED, (size_t)nfil * es));
    TRY(ensure(c, B_STATUS, (size_t)n_sys * 4));
    Run r;
    r.steps = probe_steps;
    r.dt = dt;
    r.obs_every = probe_steps;
    r.n_obs = 1;
    r.eps_over_ds = eps_over_ds;
    // the batch's filament rows on the host, for the buckets' own probes
    std::vector<double> hrows((size_t)nfil * SWIM_NPARAM);
    HIPCHK(hipMemcpyAsync(hrows.data(), params, hrows.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double* sub_rows = nullptr;
    HIPCHK(hipMalloc((void**)&sub_rows, hrows.size() * sizeof(double)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(sub_rows);
        return fail(SWIM_EHIP, "event creation failed");
    }
    const int save_graph = c->opt_graph, save_wps = c->opt_wps, save_big = c->opt_big_tpl;
    c->opt_graph = 0;
    c->opt_wps = 0;
    int rc = SWIM_OK;
    // a forward run of n systems (sizes Ns, filaments nsws, rows P on the
    // device), timed after one untimed run (first launches pay for code
    // loading)
    auto timed_on = [&](int64_t n, const int32_t* Ns, const int32_t* nsws, const double* P, float* ms) -> int {
        for (int rep = 0; rep < 2; ++rep) {
            if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) return fail(SWIM_EHIP, "event record failed");
            TRY(forward_impl(c, dtype, n, Ns, nsws, P, r, c->buf[B_OBS].p, c->buf[B_SPEED].p,
                             (int32_t*)c->buf[B_STATUS].p, nullptr, st));
        }
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipEventElapsedTime(ms, e0, e1));
        return SWIM_OK;
    };
    auto timed = [&](float* ms) -> int { return timed_on(n_sys, N, n_swim, params, ms); };
    // waves per system, one size bucket at a time (the others at their
    // current choice), then targets per lane of the large-system kernel.
    // The probe's time is the batch's throughput; a run's own speed grows
    // with its waves, and a long run's time bounds its launch (a few long
    // runs among many short ones, as in a generation whose draws mostly
    // blow up), which a short probe does not show: the most waves within
    // WPS_TIE of the fastest probe are taken.
    // Each bucket is probed alone (its systems of the batch, launched as in
    // the whole batch's calls): side by side with the others, a bucket off
    // the call's longest path would not change the call's time.
    constexpr float WPS_TIE = 1.05f;
    const int wps_cand[] = {2, 4, 8, 16};
    c->forced_launch = true;
    for (int t = 0; t <= 8; ++t) c->force_launch_tpl[t] = launch_tpl[t];
    for (int tpl = 1; tpl <= 8 && rc == SWIM_OK; ++tpl) {
        if (!has_tpl[tpl]) continue;
        std::vector<int32_t> Ns, nsws;
        std::vector<double> rows;
        int64_t f = 0;
        for (int64_t s = 0; s < n_sys; ++s) {
            const int nsw = n_swim ? n_swim[s] : 1;
            const int t0 = forward_tpl(dtype, N[s], N[s] * nsw, eps_over_ds);
            if (t0 > 0 && launch_tpl[t0] == tpl) {
                Ns.push_back(N[s]);
                nsws.push_back(nsw);
                rows.insert(rows.end(), hrows.begin() + f * SWIM_NPARAM, hrows.begin() + (f + nsw) * SWIM_NPARAM);
            }
            f += nsw;
        }
        if (hipMemcpyAsync(sub_rows, rows.data(), rows.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
            hipSuccess) {
            rc = fail(SWIM_EHIP, "upload of a bucket's rows failed");
            break;
        }
        float ms_w[4] = {};
        float best = 0.f;
        for (int k = 0; k < 4; ++k) {
            const int w = wps_cand[k];
            if (forward_lds_bytes(dtype, tpl, w) > 160 * 1024) continue;
            c->tuned_wps[dtype][tpl] = w;
            rc = timed_on((int64_t)Ns.size(), Ns.data(), nsws.data(), sub_rows, &ms_w[k]);
            if (rc != SWIM_OK) break;
            if (best == 0.f || ms_w[k] < best) best = ms_w[k];
        }
        int best_w = 16;
        for (int k = 0; k < 4; ++k)
            if (ms_w[k] > 0.f && ms_w[k] <= WPS_TIE * best) best_w = wps_cand[k];
        c->tuned_wps[dtype][tpl] = best_w;
    }
    c->forced_launch = false;
    (void)hipStreamSynchronize(st);
    (void)hipFree(sub_rows);
    // large systems: the one-sided kernel at 1, 2, 4 targets per lane and,
    // for FP32, the symmetric tile-pair step (the automatic choice, 0)
    int best_big = save_big;
    if (has_big && rc == SWIM_OK) {
        float best = 0.f;
        for (int t : {0, 1, 2, 4}) {
            if (t == 0 && dtype != SWIM_F32) continue;
            c->opt_big_tpl = t;
            float ms = 0.f;
            rc = timed(&ms);
            if (rc != SWIM_OK) break;
            if (best == 0.f || ms < best) {
                best = ms;
                best_big = t;
            }
        }
    }
    c->opt_graph = save_graph;
    c->opt_wps = save_wps;
    c->opt_big_tpl = rc == SWIM_OK ? best_big : save_big;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SWIM_OK) return rc;
    for (int tpl = 1; tpl <= 8; ++tpl) chosen[tpl - 1] = c->tuned_wps[dtype][tpl];
    chosen[8] = c->opt_big_tpl;
    return SWIM_OK;
}

int swim_tune_save(swim_ctx* c, const char* path)
{
    TRY(check_ctx(c));
    if (!path) return fail(SWIM_EINVAL, "null path");
    FILE* f = fopen(path, "w");
    if (!f) return fail(SWIM_EINVAL, "cannot write %s", path);
    fprintf(f, "swim-tune 1\n");
    for (int d = 0; d < 2; ++d) {
        fprintf(f, "wps %d", d);
        for (int t = 1; t <= 8; ++t) fprintf(f, " %d", c->tuned_wps[d][t]);
        fprintf(f, "\n");
    }
    fprintf(f, "big_tpl %d\n", c->opt_big_tpl);
    const bool ok = fclose(f) == 0;
    return ok ? SWIM_OK : fail(SWIM_EINVAL, "write error on %s", path);
}

int swim_tune_load(swim_ctx* c, const char* path)
{
    TRY(check_ctx(c));
    if (!path) return fail(SWIM_EINVAL, "null path");
    FILE* f = fopen(path, "r");
    if (!f) return fail(SWIM_EINVAL, "cannot read %s", path);
    int ver = 0, tuned[2][9] = {}, big = 0;
    bool ok = fscanf(f, " swim-tune %d", &ver) == 1 && ver == 1;
    for (int d = 0; d < 2 && ok; ++d) {
        int dd = -1;
        ok = fscanf(f, " wps %d", &dd) == 1 && dd == d;
        for (int t = 1; t <= 8 && ok; ++t) {
            ok = fscanf(f, " %d", &tuned[d][t]) == 1;
            const int w = tuned[d][t];
            ok = ok && (w == 0 || w == 1 || w == 2 || w == 4 || w == 8 || w == 16);
        }
    }
    ok = ok && fscanf(f, " big_tpl %d", &big) == 1 && (big == 0 || big == 1 || big == 2 || big == 4);
    fclose(f);
    if (!ok) return fail(SWIM_EINVAL, "%s is not a tune file of this library", path);
    for (int d = 0; d < 2; ++d)
        for (int t = 1; t <= 8; ++t) c->tuned_wps[d][t] = tuned[d][t];
    c->opt_big_tpl = big;
    return SWIM_OK;
}

}  // extern "C"


// ==========================================================================
// TMCMC (Sec. 2.3, Algorithm TMCMC): transitional Markov chain Monte Carlo
// over the batched forward model with the Gaussian likelihood of eqs.
// (likelihood)-(fitness), Sigma = sigma^2 I, sigma the fourth parameter.
// The host takes the stage decisions in FP64 (tempering exponent, weights,
// covariance, resampling, Metropolis acceptance); every likelihood is a
// forward run plus k_gauss_loglik on the device, one batched launch per
// Metropolis step across all chains.  Random streams (Philox, key = seed):
// prior stream 0 (abc_prior_draw); resampling draw k of stage j: stream
// 1000 + 2j, index k, draw 0; chain c, step s (1-based) of stage j: stream
// 1001 + 2j, index c, draws 3(s-1) .. 3(s-1)+2 (Box-Muller pairs (u0, u1),
// (u2, u3); u4 decides acceptance).
// ==========================================================================
int tmcmc_loglik(swim_ctx* c, int32_t dtype, int64_t n, int32_t n_obs, const void* obs, const double* data,
                 const double* sigma, const int32_t* status, double* logl, void* stream)
{
    TRY(check_ctx(c));
    TRY(check_dtype(dtype));
    if (n < 0 || n_obs < 1 || (n > 0 && (!obs || !data || !sigma || !status || !logl)))
        return fail(SWIM_EINVAL, "bad log-likelihood arguments");
    HIPCHK(launch_gauss_loglik(dtype, n, n_obs, obs, data, sigma, status, logl, pick(c, stream)));
    return SWIM_OK;
}

namespace {
constexpr int TM_D = 4;          // (alpha, S_b, S_s, sigma)
constexpr int TM_BISECT = 80;    // bisection steps of the tempering increment

// coefficient of variation (population standard deviation over mean) of the
// weights exp(dq (l - lmax)) over the finite log-likelihoods
double tm_weight_cv(const std::vector<double>& l, double lmax, double dq)
{
    double s = 0.0;
    int64_t k = 0;
    for (double v : l)
        if (std::isfinite(v)) {
            s += std::exp(dq * (v - lmax));
            ++k;
        }
    const double m = s / (double)k;
    double ss = 0.0;
    for (double v : l)
        if (std::isfinite(v)) {
            const double d = std::exp(dq * (v - lmax)) - m;
            ss += d * d;
        }
    return std::sqrt(ss / (double)k) / m;
}

bool chol_d(const double* A, double* L, int d)
{
    for (int i = 0; i < d * d; ++i) L[i] = 0.0;
    for (int j = 0; j < d; ++j) {
        double s = A[d * j + j];
        for (int k = 0; k < j; ++k) s -= L[d * j + k] * L[d * j + k];
        if (!(s > 0)) return false;
        L[d * j + j] = std::sqrt(s);
        for (int i = j + 1; i < d; ++i) {
            double t = A[d * i + j];
            for (int k = 0; k < j; ++k) t -= L[d * i + k] * L[d * j + k];
            L[d * i + j] = t / L[d * j + j];
        }
    }
    return true;
}
}  // namespace

// The TMCMC stages over D <= TM_D parameters (the first D of the four
// normals of each chain step are used).  evaluate(theta, k, logl) returns
// the log-likelihoods of k parameter rows of D values.
template <typename Eval>
int tmcmc_core(int D, const tmcmc_opts* o, int64_t n, uint64_t seed, Eval&& evaluate, double* theta_out,
               double* logl_out, double* q_out, int32_t* n_stages_out, double* log_evidence_out, int64_t* accepted_out)
{
    std::vector<double> theta((size_t)n * D), logl((size_t)n);
    TRY(abc_prior_draw(seed, n, D, o->lo, o->hi, theta.data()));
    TRY(evaluate(theta.data(), n, logl.data()));
    q_out[0] = 0.0;
    double q = 0.0, log_ev = 0.0;
    int stage_no = 0;
    std::vector<double> w((size_t)n), cdf((size_t)n), nth((size_t)n * D), nll((size_t)n);
    std::vector<int64_t> counts((size_t)n);
    for (; stage_no < o->max_stages && q < 1.0; ++stage_no) {
        double lmax = -INFINITY;
        for (double v : logl)
            if (std::isfinite(v)) lmax = std::max(lmax, v);
        if (!std::isfinite(lmax)) return fail(SWIM_EINVAL, "no sample has a finite likelihood");
        // tempering increment: the largest dq with weight CV <= cv_target
        double dq;
        if (tm_weight_cv(logl, lmax, 1.0 - q) <= o->cv_target) {
            dq = 1.0 - q;
        } else {
            double lo = 0.0, hi = 1.0 - q;
            for (int it = 0; it < TM_BISECT; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (tm_weight_cv(logl, lmax, mid) > o->cv_target)
                    hi = mid;
                else
                    lo = mid;
            }
            dq = lo;
        }
        const double q_next = (dq == 1.0 - q) ? 1.0 : q + dq;
        dq = q_next - q;  // the increment the weights use: from the rounded q_next
        // weights, S_j, weighted mean and covariance
        double W = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            w[i] = std::isfinite(logl[i]) ? std::exp(dq * (logl[i] - lmax)) : 0.0;
            W += w[i];
        }
        log_ev += dq * lmax + std::log(W / (double)n);
        double mu[TM_D] = {}, cov[TM_D * TM_D] = {}, L[TM_D * TM_D];  // D <= TM_D used
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < D; ++d) mu[d] += (w[i] / W) * theta[D * i + d];
        for (int64_t i = 0; i < n; ++i) {
            const double wb = w[i] / W;
            for (int d = 0; d < D; ++d)
                for (int e = 0; e < D; ++e)
                    cov[D * d + e] += wb * (theta[D * i + d] - mu[d]) * (theta[D * i + e] - mu[e]);
        }
        const double b2 = o->cov_scale * o->cov_scale;
        for (int i = 0; i < D * D; ++i) cov[i] *= b2;
        if (!chol_d(cov, L, D)) {
            for (int d = 0; d < D; ++d) cov[D * d + d] += 1e-12 * (o->hi[d] - o->lo[d]) * (o->hi[d] - o->lo[d]);
            if (!chol_d(cov, L, D)) return fail(SWIM_EINVAL, "proposal covariance is not positive definite");
        }
        // resampling: n multinomial draws by the normalized weights
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            acc += w[i] / W;
            cdf[i] = acc;
            counts[i] = 0;
        }
        for (int64_t k = 0; k < n; ++k) {
            double u[2];
            uniforms2(seed, 1000u + 2u * (uint32_t)stage_no, (uint64_t)k, 0, u);
            int64_t j = std::upper_bound(cdf.begin(), cdf.end(), u[0] * cdf.back()) - cdf.begin();
            if (j >= n) j = n - 1;
            ++counts[j];
        }
        // Metropolis chains, one per drawn sample, stepped together
        std::vector<int64_t> start, len, off;
        int64_t maxlen = 0, pos = 0;
        for (int64_t i = 0; i < n; ++i)
            if (counts[i]) {
                start.push_back(i);
                len.push_back(counts[i]);
                off.push_back(pos);
                pos += counts[i];
                maxlen = std::max(maxlen, counts[i]);
            }
        const int64_t nc = (int64_t)start.size();
        std::vector<double> cur((size_t)nc * D), lcur((size_t)nc), prop, uacc, lprop;
        std::vector<int64_t> act;
        for (int64_t ch = 0; ch < nc; ++ch) {
            for (int d = 0; d < D; ++d) cur[D * ch + d] = theta[D * start[ch] + d];
            lcur[ch] = logl[start[ch]];
        }
        int64_t accepted = 0;
        const uint32_t cstream = 1001u + 2u * (uint32_t)stage_no;
        for (int64_t s = 1; s <= maxlen; ++s) {
            act.clear();
            for (int64_t ch = 0; ch < nc; ++ch)
                if (len[ch] >= s) act.push_back(ch);
            const int64_t na = (int64_t)act.size();
            prop.resize((size_t)na * D);
            uacc.resize((size_t)na);
            std::vector<char> inbox((size_t)na);
            std::vector<double> batch;
            for (int64_t a = 0; a < na; ++a) {
                const int64_t ch = act[a];
                double u01[2], u23[2], u45[2], z[4];
                const uint32_t base = 3u * (uint32_t)(s - 1);
                uniforms2(seed, cstream, (uint64_t)ch, base, u01);
                uniforms2(seed, cstream, (uint64_t)ch, base + 1, u23);
                uniforms2(seed, cstream, (uint64_t)ch, base + 2, u45);
                box_muller(u01[0], u01[1], &z[0], &z[1]);
                box_muller(u23[0], u23[1], &z[2], &z[3]);
                uacc[a] = u45[0];
                bool in = true;
                for (int d = 0; d < D; ++d) {
                    double v = cur[D * ch + d];
                    for (int e = 0; e <= d; ++e) v += L[D * d + e] * z[e];
                    prop[D * a + d] = v;
                    in = in && v >= o->lo[d] && v <= o->hi[d];
                }
                inbox[a] = in;
                if (in) batch.insert(batch.end(), &prop[D * a], &prop[D * a] + D);
            }
            const int64_t nb = (int64_t)batch.size() / D;
            lprop.assign((size_t)nb, -INFINITY);
            TRY(evaluate(batch.data(), nb, lprop.data()));
            int64_t bi = 0;
            for (int64_t a = 0; a < na; ++a) {
                const int64_t ch = act[a];
                if (inbox[a]) {
                    const double lp = lprop[bi++];
                    if (std::log(uacc[a]) < q_next * (lp - lcur[ch])) {
                        for (int d = 0; d < D; ++d) cur[D * ch + d] = prop[D * a + d];
                        lcur[ch] = lp;
                        ++accepted;
                    }
                }
                const int64_t at = off[ch] + s - 1;
                for (int d = 0; d < D; ++d) nth[D * at + d] = cur[D * ch + d];
                nll[at] = lcur[ch];
            }
        }
        theta.swap(nth);
        logl.swap(nll);
        nth.resize((size_t)n * D);
        nll.resize((size_t)n);
        accepted_out[stage_no] = accepted;
        q = q_next;
        q_out[stage_no + 1] = q;
    }
    memcpy(theta_out, theta.data(), theta.size() * 8);
    memcpy(logl_out, logl.data(), logl.size() * 8);
    *n_stages_out = stage_no;
    *log_evidence_out = log_ev;
    return SWIM_OK;
}

int tmcmc_run(swim_ctx* c, const abc_model* m, const tmcmc_opts* o, const double* data, int32_t n_obs, int32_t N,
              int64_t n, uint64_t seed, double* theta_out, double* logl_out, double* q_out, int32_t* n_stages_out,
              double* log_evidence_out, int64_t* accepted_out, int64_t* runs_out, double* seconds_out)
{
    TRY(check_ctx(c));
    if (!m || !o || !data || !theta_out || !logl_out || !q_out || !n_stages_out || !log_evidence_out || !accepted_out)
        return fail(SWIM_EINVAL, "null argument");
    TRY(check_dtype(m->dtype));
    if (n < 2) return fail(SWIM_EINVAL, "n must be >= 2");
    if (m->obs_every < 1 || n_obs != m->steps / m->obs_every) return fail(SWIM_EINVAL, "n_obs must equal steps/obs_every");
    if (o->max_stages < 1) return fail(SWIM_EINVAL, "max_stages must be >= 1");
    if (!(o->cv_target > 0 && std::isfinite(o->cv_target))) return fail(SWIM_EINVAL, "cv_target must be > 0");
    if (!(o->cov_scale > 0 && std::isfinite(o->cov_scale))) return fail(SWIM_EINVAL, "cov_scale must be > 0");
    for (int d = 0; d < TM_D; ++d)
        if (!(std::isfinite(o->lo[d]) && std::isfinite(o->hi[d]) && o->hi[d] > o->lo[d]))
            return fail(SWIM_EINVAL, "bad prior box");
    if (!(o->lo[3] > 0)) return fail(SWIM_EINVAL, "the prior box of sigma must be positive");
    {
        const int32_t Nchk = N;
        TRY(check_run(1, &Nchk, nullptr, m->steps, m->dt, m->obs_every, m->eps_over_ds));
    }
    hipStream_t st = c->stream;
    const size_t es = m->dtype == SWIM_F32 ? 4 : 8;
    Run r;
    r.steps = m->steps;
    r.dt = m->dt;
    r.obs_every = m->obs_every;
    r.n_obs = n_obs;
    r.eps_over_ds = m->eps_over_ds;
    double t_eval = 0.0;
    int64_t runs = 0;
    // log-likelihoods of k parameter points (rows of TM_D), one batched
    // forward launch and one likelihood launch
    std::vector<double> rows, sig;
    std::vector<int32_t> Nv;
    auto evaluate = [&](const double* th, int64_t k, double* ll) -> int {
        if (k == 0) return SWIM_OK;
        const auto t0 = std::chrono::steady_clock::now();
        rows.assign((size_t)k * SWIM_NPARAM, 0.0);
        sig.resize((size_t)k);
        Nv.assign((size_t)k, N);
        for (int64_t i = 0; i < k; ++i) {
            double* P = &rows[(size_t)i * SWIM_NPARAM];
            P[0] = th[TM_D * i];
            P[1] = th[TM_D * i + 1];
            P[2] = th[TM_D * i + 2];
            P[3] = m->b;
            P[4] = m->omega;
            P[5] = m->k;
            sig[(size_t)i] = th[TM_D * i + 3];
        }
        TRY(ensure(c, B_OBS, (size_t)k * n_obs * 2 * es));
        TRY(ensure(c, B_SPEED, (size_t)k * es));
        TRY(ensure(c, B_STATUS, (size_t)k * 4));
        TRY(ensure(c, B_SIGMA, (size_t)k * 8));
        TRY(ensure(c, B_LOGL, (size_t)k * 8));
        TRY(begin_uploads(c, rows.size() * 8 + sig.size() * 8 + (size_t)n_obs * 16));
        TRY(stage(c, rows.data(), rows.size() * 8, B_PARAMS, st));
        TRY(stage(c, sig.data(), sig.size() * 8, B_SIGMA, st));
        TRY(stage(c, data, (size_t)n_obs * 16, B_DATA, st));
        TRY(end_uploads(c, st));
        const int save_graph = c->opt_graph;
        if (!m->use_graph) c->opt_graph = 0;
        const int frc = forward_impl(c, m->dtype, k, Nv.data(), nullptr, (const double*)c->buf[B_PARAMS].p, r,
                                     c->buf[B_OBS].p, c->buf[B_SPEED].p, (int32_t*)c->buf[B_STATUS].p, nullptr, st);
        c->opt_graph = save_graph;
        TRY(frc);
        HIPCHK(launch_gauss_loglik(m->dtype, k, n_obs, c->buf[B_OBS].p, (const double*)c->buf[B_DATA].p,
                                   (const double*)c->buf[B_SIGMA].p, (const int32_t*)c->buf[B_STATUS].p,
                                   (double*)c->buf[B_LOGL].p, st));
        HIPCHK(hipMemcpyAsync(ll, c->buf[B_LOGL].p, (size_t)k * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        runs += k;
        t_eval += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return SWIM_OK;
    };
    TRY(tmcmc_core(TM_D, o, n, seed, evaluate, theta_out, logl_out, q_out, n_stages_out, log_evidence_out,
                   accepted_out));
    if (runs_out) *runs_out = runs;
    if (seconds_out) *seconds_out = t_eval;
    return SWIM_OK;
}

// TMCMC over the full sperm model (Sec. 4): the stages of tmcmc_core; each
// likelihood is a sperm forward run, the observables of model->kind and the
// two-level Gaussian likelihood on the device.
int tmcmc_sperm_run(swim_ctx* c, const sperm_tmcmc_model* m, const double* swim_rows, const tmcmc_opts* o,
                    const double* data, int32_t n_obs, int64_t n, uint64_t seed, double* theta_out, double* logl_out,
                    double* q_out, int32_t* n_stages_out, double* log_evidence_out, int64_t* accepted_out,
                    int64_t* runs_out, double* seconds_out)
{
    TRY(check_ctx(c));
    if (!m || !o || !swim_rows || !data || !theta_out || !logl_out || !q_out || !n_stages_out || !log_evidence_out ||
        !accepted_out)
        return fail(SWIM_EINVAL, "null argument");
    TRY(check_dtype(m->dtype));
    TRY(sperm_check(&m->shape, m->steps, m->dt, m->obs_every));
    const int d = m->n_theta, ns = m->n_sigma, nf = d - ns;
    if (d < 2 || d > TM_D) return fail(SWIM_EINVAL, "n_theta must be in [2, 4]");
    if (ns < 1 || ns > 2 || nf < 1) return fail(SWIM_EINVAL, "n_sigma must be 1 or 2, with at least one model field");
    for (int i = 0; i < nf; ++i)
        if (m->field[i] < 0 || m->field[i] >= SWIM_SP_NPARAM) return fail(SWIM_EINVAL, "bad field index");
    if (m->kind != SWIM_OBS_HEAD_VELOCITY && m->kind != SWIM_OBS_PAIR_DISTANCES)
        return fail(SWIM_EINVAL, "unknown observable kind");
    if (m->kind == SWIM_OBS_PAIR_DISTANCES && m->shape.n_swim < 2) return fail(SWIM_EINVAL, "distances need two swimmers");
    if (!(m->beta[0] > 0 && m->beta[1] > 0 && std::isfinite(m->beta[0]) && std::isfinite(m->beta[1])))
        return fail(SWIM_EINVAL, "beta must be finite and > 0");
    if (m->obs_every < 1 || n_obs != m->steps / m->obs_every) return fail(SWIM_EINVAL, "n_obs must equal steps/obs_every");
    if (n < 2) return fail(SWIM_EINVAL, "n must be >= 2");
    if (o->max_stages < 1) return fail(SWIM_EINVAL, "max_stages must be >= 1");
    if (!(o->cv_target > 0 && std::isfinite(o->cv_target))) return fail(SWIM_EINVAL, "cv_target must be > 0");
    if (!(o->cov_scale > 0 && std::isfinite(o->cov_scale))) return fail(SWIM_EINVAL, "cov_scale must be > 0");
    for (int k = 0; k < d; ++k)
        if (!(std::isfinite(o->lo[k]) && std::isfinite(o->hi[k]) && o->hi[k] > o->lo[k]))
            return fail(SWIM_EINVAL, "bad prior box");
    for (int k = nf; k < d; ++k)
        if (!(o->lo[k] >= 0)) return fail(SWIM_EINVAL, "the prior box of a noise level must be >= 0");
    const int nsw = m->shape.n_swim;
    const size_t es = m->dtype == SWIM_F32 ? 4 : 8;
    const double dt_obs = m->dt * (double)m->obs_every;
    hipStream_t st = c->stream;
    double t_eval = 0.0;
    int64_t runs = 0;
    std::vector<double> rows, sw, sig;
    auto evaluate = [&](const double* th, int64_t k, double* ll) -> int {
        if (k == 0) return SWIM_OK;
        const auto t0 = std::chrono::steady_clock::now();
        rows.resize((size_t)k * SWIM_SP_NPARAM);
        sw.resize((size_t)k * nsw * 3);
        sig.resize((size_t)k * 2);
        for (int64_t i = 0; i < k; ++i) {
            double* P = &rows[(size_t)i * SWIM_SP_NPARAM];
            for (int f = 0; f < SWIM_SP_NPARAM; ++f) P[f] = m->sys_row[f];
            for (int f = 0; f < nf; ++f) P[m->field[f]] = th[(size_t)d * i + f];
            memcpy(&sw[(size_t)i * nsw * 3], swim_rows, sizeof(double) * nsw * 3);
            const double ga = th[(size_t)d * i + nf], gb = th[(size_t)d * i + d - 1];
            sig[2 * i] = ga * m->beta[0];
            sig[2 * i + 1] = gb * m->beta[1];
        }
        TRY(ensure(c, B_SP_HEAD, (size_t)k * nsw * (n_obs + 1) * 2 * es));
        TRY(ensure(c, B_SP_TAIL, (size_t)k * nsw * (n_obs + 1) * 2 * es));
        TRY(ensure(c, B_SP_G, (size_t)k * n_obs * 2 * 8));
        TRY(ensure(c, B_STATUS, (size_t)k * 4));
        TRY(ensure(c, B_LOGL, (size_t)k * 8));
        TRY(begin_uploads(c, rows.size() * 8 + sw.size() * 8 + sig.size() * 8 + (size_t)n_obs * 16));
        TRY(stage(c, rows.data(), rows.size() * 8, B_PARAMS, st));
        TRY(stage(c, sw.data(), sw.size() * 8, B_SP_SW, st));
        TRY(stage(c, sig.data(), sig.size() * 8, B_SP_SIG, st));
        TRY(stage(c, data, (size_t)n_obs * 16, B_DATA, st));
        TRY(end_uploads(c, st));
        TRY(sperm_forward_impl(c, m->dtype, k, m->shape, (const double*)c->buf[B_PARAMS].p,
                               (const double*)c->buf[B_SP_SW].p, m->steps, m->dt, m->obs_every, c->buf[B_SP_HEAD].p,
                               c->buf[B_SP_TAIL].p, (int32_t*)c->buf[B_STATUS].p, st));
        HIPCHK(launch_sperm_observables(m->dtype, m->kind, k, nsw, n_obs, dt_obs, c->buf[B_SP_HEAD].p,
                                        c->buf[B_SP_TAIL].p, (const int32_t*)c->buf[B_STATUS].p,
                                        (double*)c->buf[B_SP_G].p, st));
        HIPCHK(launch_gauss_loglik2(k, n_obs, (const double*)c->buf[B_SP_G].p, (const double*)c->buf[B_DATA].p,
                                    (const double*)c->buf[B_SP_SIG].p, (const int32_t*)c->buf[B_STATUS].p,
                                    (double*)c->buf[B_LOGL].p, st));
        HIPCHK(hipMemcpyAsync(ll, c->buf[B_LOGL].p, (size_t)k * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        runs += k;
        t_eval += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return SWIM_OK;
    };
    TRY(tmcmc_core(d, o, n, seed, evaluate, theta_out, logl_out, q_out, n_stages_out, log_evidence_out,
                   accepted_out));
    if (runs_out) *runs_out = runs;
    if (seconds_out) *seconds_out = t_eval;
    return SWIM_OK;
}

// Host runtime of libaap.so: parameter validation, workspace layout, launch
// sequence of a step, state transfer, measurement readout.  Implements the C
// ABI declared in include/aap.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "aap.h"
#include "aap_internal.h"

using namespace aap;

// ---------------------------------------------------------------------------
// Scratch of aap_fields_noalloc: the integer field accumulators
// (fields_scratch_bytes(G) bytes) for grids up to kNoAllocMaxG, as a static
// device array.  Each GPU the library runs on holds its own copy until the
// process ends.  Host code never passes the name to a kernel: the device
// address of each GPU's copy comes from hipGetSymbolAddress, called once per
// device with that device current, and is kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
constexpr int kNoAllocMaxG = 512;
constexpr size_t kNoAllocScratchBytes = (size_t)kNoAllocMaxG * kNoAllocMaxG * (4 + 8 + 8);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define AAP_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(AAP_EHIP, "%s: %s", #call, hipGetErrorString(e_));     \
    } while (0)

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on GPU dev (looked up on first use, with
// dev made current for the lookup and the caller's device restored).
int noalloc_scratch(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(AAP_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess)
            return fail(AAP_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        if (!p) return fail(AAP_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AAP_OK;
}

// Cells per axis: the largest M whose cell side L/M exceeds R by the
// relative margin 2^-20 ("a little larger than R", Sec. 3.2), so the 3x3
// scan reaches every pair with d <= R whatever the rounding of the cell ids.
int cells_per_axis(double L, double R) {
    const double m = std::floor(L / (R * (1.0 + 0x1p-20)));
    if (!(m >= 1.0)) return 0;
    if (m > 2147483647.0) return 2147483647;
    return (int)m;
}

struct Layout {
    int Mx = 0, My = 0;
    uint64_t ncells = 0;
    size_t off_candA = 0, off_oriA = 0, off_candB = 0, off_oriB = 0, off_kslot = 0,
           off_key = 0, off_count = 0, off_start = 0, off_start2 = 0, off_status = 0, off_ticket = 0, off_obs = 0,
           off_acc = 0, off_tiles = 0, off_hbins = 0, off_hacc = 0, off_series = 0, off_dbg_n = 0, off_dbg_C = 0, off_dbg_S = 0,
           off_h = 0, off_err = 0, off_toff = 0, off_dstep = 0;
    size_t bytes = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int validate(const aap_params* p, Layout* lay) {
    if (!p) return fail(AAP_EINVAL, "params is NULL");
    if (p->N < 1 || p->N > 0xFFFFFFFFull)
        return fail(AAP_EINVAL, "N must be in [1, 2^32-1] (got %llu)", (unsigned long long)p->N);
    if (!(std::isfinite(p->Lx) && std::isfinite(p->Ly) && std::isfinite(p->R)) ||
        !(p->Lx > 0 && p->Ly > 0 && p->R > 0))
        return fail(AAP_EINVAL, "Lx, Ly, R must be finite and > 0");
    const double Lx = (double)(float)p->Lx, Ly = (double)(float)p->Ly;
    if (!(Lx > 0 && Ly > 0 && std::isfinite(Lx) && std::isfinite(Ly)))
        return fail(AAP_EINVAL, "box sides do not fit binary32");
    const int Mx = cells_per_axis(Lx, p->R), My = cells_per_axis(Ly, p->R);
    if (Mx < 3 || My < 3)
        return fail(AAP_EINVAL, "box must hold >= 3 cells of side > R per axis (Mx=%d, My=%d)",
                    Mx, My);
    if ((uint64_t)Mx * (uint64_t)My > 0x7FFFFFFFull)
        return fail(AAP_EINVAL, "too many cells (%d x %d)", Mx, My);
    if (p->rule != AAP_RULE_VM && p->rule != AAP_RULE_LANGEVIN && p->rule != AAP_RULE_NVM)
        return fail(AAP_EINVAL, "unknown rule %d", p->rule);
    if (p->rule == AAP_RULE_LANGEVIN ? (p->order < 1 || p->order > kMaxOrder) : p->order != 1)
        return fail(AAP_EINVAL, "interaction order %d: must be 1 for the Vicsek rules, "
                    "1..%d for the Langevin rule", p->order, kMaxOrder);
    if (!(std::isfinite(p->v) && std::isfinite(p->eta) && std::isfinite(p->omega) &&
          std::isfinite(p->gamma) && std::isfinite(p->dt)))
        return fail(AAP_EINVAL, "v, eta, omega, gamma, dt must be finite");
    if (p->eta < 0) return fail(AAP_EINVAL, "eta must be >= 0");
    if (p->rule == AAP_RULE_LANGEVIN && !(p->dt > 0))
        return fail(AAP_EINVAL, "dt must be > 0 for the Langevin rule");
    const double disp = std::fabs(p->rule != AAP_RULE_LANGEVIN ? p->v : p->v * p->dt);
    if (!(disp < 0.5 * std::min(Lx, Ly)))
        return fail(AAP_EINVAL, "displacement per step must be < min(L)/2");
    if (p->weights && p->weight_len < 1)
        return fail(AAP_EINVAL, "weight_len must be >= 1 when weights are given");
    if (p->weights) {
        for (int k = 0; k < p->weight_len; ++k)
            if (!std::isfinite(p->weights[k]))
                return fail(AAP_EINVAL, "weights[%d] is not finite", k);
    }
    if ((p->bins_theta == 0) != (p->bins_n == 0) || p->bins_theta < 0 || p->bins_n < 0 ||
        p->bins_theta > kHistMaxBins || p->bins_n > kHistMaxBins)
        return fail(AAP_EINVAL, "histogram bins must both be 0 or both in [1, %d]", kHistMaxBins);
    if (!lay) return AAP_OK;

    Layout L;
    L.Mx = Mx;
    L.My = My;
    L.ncells = (uint64_t)Mx * My;
    const size_t N = (size_t)p->N;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.off_candA = take(N * sizeof(Cand));
    L.off_oriA = take(N * sizeof(Ori));
    // kCandPad records past the end: candidate batches may read beyond the last
    // window (values unused)
    L.off_candB = take((N + kCandPad) * sizeof(Cand));
    L.off_oriB = take(N * sizeof(Ori));
    L.off_kslot = take(N * sizeof(uint2));
    L.off_key = take(N * 4);
    L.off_count = take(L.ncells * 4);
    L.off_start = take((L.ncells + 1) * 4);
    L.off_start2 = take((L.ncells + 1) * 4);
    L.off_status = take((size_t)scan_blocks((uint32_t)L.ncells) * 8);
    L.off_ticket = take(8);
    L.off_tiles = take((size_t)sort_blocks((uint32_t)L.ncells) * kTileSpread * 2 * 4);   // two buffers
    L.off_toff = take((size_t)sort_blocks((uint32_t)L.ncells) * 4);
    L.off_obs = take((size_t)kObsSlots * kObsWords * 8);
    L.off_hacc = take((size_t)(p->bins_theta + p->bins_n) * 8 + 8);   // zeroed with the above
    L.off_acc = take(16 * 8);
    L.off_series = take((size_t)kSeriesCap * 8);
    L.off_hbins = take(p->bins_theta > 0 ? N * 4 : 4);
    L.off_dbg_n = take(N * 4);
    L.off_dbg_C = take(N * 4);
    L.off_dbg_S = take(N * 4);
    L.off_h = take((size_t)(p->weights ? p->weight_len : 1) * 4);
    L.off_err = take(4);
    L.off_dstep = take(4);
    L.bytes = o;
    *lay = L;
    return AAP_OK;
}

struct TimerSlot {
    const char* name;
    std::vector<hipEvent_t> ev;   // start, stop pairs not yet read
    double total_ms = 0.0;
    int64_t launches = 0;
};

// binary32 bounds lo <= R^2 - m and hi >= R^2 + m (rounded outward)
void prefilter_band(double R2, double m, float& lo, float& hi) {
    lo = (float)(R2 - m);
    hi = (float)(R2 + m);
    if ((double)lo > R2 - m) lo = std::nextafter(lo, -INFINITY);
    if ((double)hi < R2 + m) hi = std::nextafter(hi, INFINITY);
}

}  // namespace

namespace aap {
int set_error(int code, const char* msg) {
    g_err = msg;
    return code;
}
}  // namespace aap

struct aap_sim {
    aap_params p;
    Layout lay;
    hipStream_t stream = nullptr;
    int device = 0;
    unsigned char* ws = nullptr;
    Cand* candA = nullptr;      // state, in the (cell, id) order of the last step
    Ori* oriA = nullptr;
    Cand* candB = nullptr;      // state binned by its current cells
    Ori* oriB = nullptr;
    uint2* kslot = nullptr;     // (cell, slot in cell) per particle of candA (fresh state)
    uint32_t* key = nullptr;    // next cell per particle of candA
    uint32_t* count = nullptr;  // histogram of a fresh state's cells
    uint32_t* startbuf[2] = {nullptr, nullptr};   // cell starts: current, and the next sort's
    int cur = 0;                // startbuf[cur] describes candB (and the order of candA)
    bool fresh = true;          // candA is not in cell order: sort with k_scan + k_scatter
    uint32_t rows_per_step = 1; // cell rows a particle can cross in one step
    unsigned long long* status = nullptr;
    unsigned long long* ticket = nullptr;
    uint32_t* tiles[2] = {nullptr, nullptr};  // arrivals per k_sort tile, two buffers
    uint32_t* tile_off = nullptr;  // per tile: arrivals before it (large grids)
    int tcur = 0;               // the buffer the next neighbour kernel fills
    long long* obs_slots = nullptr;
    double* acc = nullptr;
    double* series = nullptr;
    uint32_t* dbg_n = nullptr;
    float* dbg_C = nullptr;
    float* dbg_S = nullptr;
    float* htab = nullptr;
    std::vector<double> weights;  // host copy of the weight table (checkpoints compare it)
    uint32_t* hbins = nullptr;    // per-particle histogram bins of a measured step
    unsigned long long* hacc = nullptr;   // angle counts [bins_theta], then n counts [bins_n]
    uint32_t* err = nullptr;
    Geom g;
    Model m;
    float r2_lo = 0.f, r2_hi = 0.f, r2_lo_edge = 0.f, r2_hi_edge = 0.f;
    uint64_t step = 0;
    bool debug = false;
    bool debug_valid = false;
    bool obs_pending = false;   // the last neighbour launch measured a state not yet folded
    int obs_slot = -1;          // series slot of that state (-1: not recorded)
    bool timing = false;         // timing enabled
    bool timing_now = false;     // this step's launches carry events
    int timing_every = 0;
    int64_t timing_count = 0;    // steps since timing was enabled
    std::vector<TimerSlot> timers;
    std::vector<hipEvent_t> event_pool;
    uint32_t* d_step = nullptr;   // the step captured neighbour kernels read (the sort advances it)
    hipStream_t cap = nullptr;    // private stream for graph capture
    int graph_steps = 0;          // steps per captured graph (0: every step launched)
    bool capturing = false;       // one_step is recording into a graph
    hipGraph_t graph[2][2][2] = {};       // [measure][cur][tcur] at the graph's start
    hipGraphExec_t exec[2][2][2] = {};
};

namespace {

enum { kTScan = 0, kTScatter, kTNbr, kTSort, kTCount };

hipEvent_t take_event(aap_sim* s) {
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    // default events: of the flags measured on timed launches of k_nbr and
    // k_sort against the profiler's durations, they add the least (~4 us per
    // launch; without system fences 4.5-9 us, with device-scope release 4.4-5.5)
    if (hipEventCreateWithFlags(&e, hipEventDefault) != hipSuccess) return nullptr;
    return e;
}

// Folds recorded (start, stop) event pairs into the per-kernel totals.  With
// all == false only the older half of each list is folded, waiting on its
// last event alone, so the stream keeps the newer launches queued and the
// device does not idle while a long timed run is drained.
int drain_timers(aap_sim* s, bool all = true) {
    if (all) AAP_HIP(hipStreamSynchronize(s->stream));
    for (auto& t : s->timers) {
        const size_t upto = all ? t.ev.size() : (t.ev.size() / 4) * 2;
        if (upto < 2) continue;
        if (!all) AAP_HIP(hipEventSynchronize(t.ev[upto - 1]));
        for (size_t k = 0; k + 1 < upto; k += 2) {
            float ms = 0.f;
            AAP_HIP(hipEventElapsedTime(&ms, t.ev[k], t.ev[k + 1]));
            t.total_ms += ms;
            t.launches += 1;
            s->event_pool.push_back(t.ev[k]);
            s->event_pool.push_back(t.ev[k + 1]);
        }
        t.ev.erase(t.ev.begin(), t.ev.begin() + upto);
    }
    return AAP_OK;
}

// An event pair for one timed launch, taken from the pool when timing is on
// (both null otherwise); done() files it under its kernel.
struct TimedLaunch {
    aap_sim* s;
    int which;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TimedLaunch(aap_sim* s_, int w) : s(s_), which(w) {
        if (s->timing_now) {
            e0 = take_event(s);
            e1 = e0 ? take_event(s) : nullptr;
            if (!e1 && e0) {
                s->event_pool.push_back(e0);
                e0 = nullptr;
            }
        }
    }
    void done() {
        if (e0 && e1) {
            s->timers[which].ev.push_back(e0);
            s->timers[which].ev.push_back(e1);
        }
    }
};

int check_device_error(aap_sim* s) {
    uint32_t e = 0;
    AAP_HIP(hipMemcpyAsync(&e, s->err, 4, hipMemcpyDeviceToHost, s->stream));
    AAP_HIP(hipStreamSynchronize(s->stream));
    if (e) return fail(AAP_EHIP, "internal cell-list inconsistency (error bits 0x%x)", e);
    return AAP_OK;
}

// Cell ids, histogram and slots of the state in candA/oriA (after init or a
// state given by the caller).
int rebuild_cells(aap_sim* s) {
    const uint32_t N = (uint32_t)s->p.N;
    AAP_HIP(launch_fill_u32(s->count, s->lay.ncells, 0u, s->stream));
    AAP_HIP(launch_prepare(s->candA, s->oriA, s->kslot, s->key, s->count, N, s->g, s->m.order,
                           s->stream));
    AAP_HIP(launch_fill_u32(s->tiles[s->tcur],
                            (uint64_t)sort_blocks((uint32_t)s->lay.ncells) * kTileSpread, 0u,
                            s->stream));
    s->fresh = true;
    return AAP_OK;
}

// Folds the measured sums of the last neighbour launch, if any, into the
// accumulators (one small launch; the scan kernel does it otherwise).
int finalize_obs(aap_sim* s) {
    if (!s->obs_pending) return AAP_OK;
    AAP_HIP(launch_obs(s->obs_slots, s->acc, s->series, s->obs_slot, (uint32_t)s->p.N,
                       s->stream));
    s->obs_pending = false;
    return AAP_OK;
}

// The neighbour-kernel arguments of s for the state sorted into
// startbuf[cur], the arrivals counted into tiles[tcur].
NbrArgs nbr_args(const aap_sim* s, int cur, int tcur, bool measure, bool hist, bool debug) {
    NbrArgs a;
    a.candB = s->candB;
    a.oriB = s->oriB;
    a.start = s->startbuf[cur];
    a.candA = s->candA;
    a.oriA = s->oriA;
    a.key_out = s->key;
    a.tile_count = s->tiles[tcur];
    a.hist_bins = hist ? s->hbins : nullptr;
    a.hist_scale = (double)s->p.bins_theta / (2.0 * 3.14159265358979311600);
    a.hist_bt = (uint32_t)s->p.bins_theta;
    a.hist_bn = (uint32_t)s->p.bins_n;
    a.obs_slots = measure ? s->obs_slots : nullptr;
    a.dbg_n = debug ? s->dbg_n : nullptr;
    a.dbg_C = debug ? s->dbg_C : nullptr;
    a.dbg_S = debug ? s->dbg_S : nullptr;
    a.err = s->err;
    a.g = s->g;
    a.m = s->m;
    a.N = (uint32_t)s->p.N;
    a.step = (uint32_t)s->step;
    a.step_dev = s->capturing ? s->d_step : nullptr;
    a.r2_lo = s->r2_lo;
    a.r2_hi = s->r2_hi;
    a.r2_lo_edge = s->r2_lo_edge;
    a.r2_hi_edge = s->r2_hi_edge;
    return a;
}

// The counting-sort arguments of s for a state in the order of
// startbuf[cur] (arrivals counted in tiles[cur]), sorted into the other
// buffers.
SortArgs sort_args_of(const aap_sim* s, int cur) {
    return sort_args(s->candA, s->oriA, s->key, s->startbuf[cur], s->startbuf[1 - cur], s->candB,
                     s->oriB, (uint32_t)s->lay.ncells, (uint32_t)s->p.N, (uint32_t)s->lay.Mx,
                     (uint32_t)s->lay.My, s->rows_per_step, s->g.by ? 0 : 1, s->tiles[cur],
                     s->tiles[1 - cur], s->obs_slots, s->acc, s->series, -1, s->err);
}

int one_step(aap_sim* s, bool measure, bool record, uint32_t slot) {
    const uint32_t N = (uint32_t)s->p.N;
    s->timing_now = s->timing && (s->timing_count++ % s->timing_every) == 0;
    if (s->fresh) {
        // candA in any order: histogram from k_prepare, scan, scatter by slot
        {
            TimedLaunch tl(s, kTScan);
            AAP_HIP(launch_scan(s->count, s->startbuf[s->cur], (uint32_t)s->lay.ncells, s->status,
                                s->ticket, s->obs_slots, s->acc, s->series,
                                s->obs_pending ? 1 : 0, s->obs_slot, N, s->stream, tl.e0, tl.e1));
            tl.done();
        }
        {
            TimedLaunch tl(s, kTScatter);
            AAP_HIP(launch_scatter(s->candA, s->oriA, s->kslot, s->startbuf[s->cur], s->candB,
                                   s->oriB, N, s->err, s->stream, tl.e0, tl.e1));
            tl.done();
        }
        s->fresh = false;
    } else {
        // candA in the order of startbuf[cur]: one counting-sort kernel into
        // the other start buffer (on large grids after a scan of the tile
        // counts)
        const uint32_t nblocks = sort_blocks((uint32_t)s->lay.ncells);
        const uint32_t* toff = nullptr;
        if (nblocks >= kTileScanMin) {
            AAP_HIP(launch_tile_offsets(s->tiles[s->tcur], nblocks, s->tile_off, s->stream));
            toff = s->tile_off;
        }
        TimedLaunch tl(s, kTSort);
        AAP_HIP(launch_sort(s->candA, s->oriA, s->key, s->startbuf[s->cur], s->startbuf[1 - s->cur],
                            s->candB, s->oriB, (uint32_t)s->lay.ncells, N, (uint32_t)s->lay.Mx,
                            (uint32_t)s->lay.My, s->rows_per_step, s->g.by ? 0 : 1,
                            s->tiles[s->tcur], s->tiles[1 - s->tcur], toff, s->obs_slots, s->acc, s->series, s->obs_pending ? 1 : 0,
                            s->obs_slot, s->err, s->capturing ? s->d_step : nullptr, s->stream,
                            tl.e0, tl.e1));
        tl.done();
        s->cur = 1 - s->cur;
        s->tcur = 1 - s->tcur;
    }
    s->obs_pending = false;
    const bool hist = measure && s->p.bins_theta > 0;
    const NbrArgs a = nbr_args(s, s->cur, s->tcur, measure, hist, s->debug);
    {
        TimedLaunch tl(s, kTNbr);
        AAP_HIP(launch_nbr(a, s->stream, tl.e0, tl.e1));
        tl.done();
    }
    if (hist)
        AAP_HIP(launch_hist(s->hbins, N, (uint32_t)s->p.bins_theta, (uint32_t)s->p.bins_n,
                            s->hacc, s->hacc + s->p.bins_theta, s->stream));
    if (measure) {
        s->obs_pending = true;
        s->obs_slot = record ? (int)slot : -1;
    }
    s->debug_valid = s->debug;
    s->step += 1;
    if (s->timing && s->timers[kTNbr].ev.size() > 4096) return drain_timers(s, false);
    return AAP_OK;
}

void sim_drop_graphs(aap_sim* s) {
    for (auto& m : s->exec)
        for (auto& c : m)
            for (hipGraphExec_t& e : c) {
                if (e) (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
    for (auto& m : s->graph)
        for (auto& c : m)
            for (hipGraph_t& g : c) {
                if (g) (void)hipGraphDestroy(g);
                g = nullptr;
            }
}

// The graph of graph_steps steps (measured or not) from the current parity,
// captured on the private stream on first use: one_step records its
// launches there with the step read from d_step (which the sort advances),
// no series slot and no timing events; the host state it changes is put
// back, since nothing ran.  Its first sort folds a pending measured state
// exactly when measure is set (aap_step replays it only then).
int sim_graph(aap_sim* s, bool measure, hipGraphExec_t* out) {
    hipGraphExec_t& e = s->exec[measure ? 1 : 0][s->cur][s->tcur];
    if (!e) {
        if (!s->cap) AAP_HIP(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
        const uint64_t step0 = s->step;
        const int cur0 = s->cur, tcur0 = s->tcur, slot0 = s->obs_slot;
        const bool pend0 = s->obs_pending, dv0 = s->debug_valid;
        const int64_t tc0 = s->timing_count;
        hipStream_t st0 = s->stream;
        const hipError_t eb = hipStreamBeginCapture(s->cap, hipStreamCaptureModeRelaxed);
        if (eb != hipSuccess) return fail(AAP_EHIP, "graph capture: %s", hipGetErrorString(eb));
        s->stream = s->cap;
        s->capturing = true;
        int rc = AAP_OK;
        for (int k = 0; k < s->graph_steps && rc == AAP_OK; ++k) rc = one_step(s, measure, false, 0);
        hipGraph_t got = nullptr;
        const hipError_t ee = hipStreamEndCapture(s->cap, &got);
        s->stream = st0;
        s->capturing = false;
        s->step = step0;
        s->cur = cur0;
        s->tcur = tcur0;
        s->obs_slot = slot0;
        s->obs_pending = pend0;
        s->debug_valid = dv0;
        s->timing_count = tc0;
        if (rc || ee != hipSuccess) {
            if (got) (void)hipGraphDestroy(got);
            return rc ? rc : fail(AAP_EHIP, "graph capture: %s", hipGetErrorString(ee));
        }
        s->graph[measure ? 1 : 0][cur0][tcur0] = got;
        AAP_HIP(hipGraphInstantiate(&e, got, nullptr, nullptr, 0));
    }
    *out = e;
    return AAP_OK;
}

// Copies the current state to host, in the device's (cell, id) order.
int fetch_state(aap_sim* s, std::vector<Cand>& c, std::vector<Ori>& o) {
    const size_t N = (size_t)s->p.N;
    try {
        c.resize(N);
        o.resize(N);
    } catch (...) {
        return fail(AAP_ENOMEM, "host allocation failed");
    }
    AAP_HIP(hipMemcpyAsync(c.data(), s->candA, N * sizeof(Cand), hipMemcpyDeviceToHost,
                           s->stream));
    AAP_HIP(hipMemcpyAsync(o.data(), s->oriA, N * sizeof(Ori), hipMemcpyDeviceToHost,
                           s->stream));
    return check_device_error(s);
}

}  // namespace

extern "C" {

aap_params aap_params_default(void) {
    aap_params p;
    std::memset(&p, 0, sizeof p);
    p.N = 4096;
    p.Lx = 64.0;
    p.Ly = 64.0;
    p.R = 1.0;
    p.v = 0.5;
    p.eta = 0.3;
    p.omega = 0.0;
    p.gamma = 1.0;
    p.dt = 1.0;
    p.rule = AAP_RULE_VM;
    p.order = 1;
    p.bx = 0;
    p.by = 0;
    p.seed = 0;
    p.weights = nullptr;
    p.weight_len = 0;
    p.bins_theta = 0;
    p.bins_n = 0;
    return p;
}

int aap_workspace_bytes(const aap_params* p, size_t* bytes) {
    if (!bytes) return fail(AAP_EINVAL, "bytes is NULL");
    Layout L;
    const int rc = validate(p, &L);
    if (rc) return rc;
    *bytes = L.bytes;
    return AAP_OK;
}

int aap_create(const aap_params* p, void* d_workspace, size_t bytes, void* hip_stream,
               aap_sim** out) {
    if (!out) return fail(AAP_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    int rc = validate(p, &L);
    if (rc) return rc;
    if (!d_workspace) return fail(AAP_EINVAL, "workspace is NULL");
    if (((uintptr_t)d_workspace & 255u) != 0)
        return fail(AAP_ENOMEM, "workspace must be 256-byte aligned");
    if (bytes < L.bytes)
        return fail(AAP_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, L.bytes);

    aap_sim* s = new (std::nothrow) aap_sim();
    if (!s) return fail(AAP_ENOMEM, "host allocation failed");
    s->p = *p;
    s->p.weights = nullptr;   // copied below, not retained
    s->lay = L;
    s->stream = (hipStream_t)hip_stream;
    s->ws = (unsigned char*)d_workspace;
    s->candA = (Cand*)(s->ws + L.off_candA);
    s->oriA = (Ori*)(s->ws + L.off_oriA);
    s->candB = (Cand*)(s->ws + L.off_candB);
    s->oriB = (Ori*)(s->ws + L.off_oriB);
    s->kslot = (uint2*)(s->ws + L.off_kslot);
    s->key = (uint32_t*)(s->ws + L.off_key);
    s->count = (uint32_t*)(s->ws + L.off_count);
    s->startbuf[0] = (uint32_t*)(s->ws + L.off_start);
    s->startbuf[1] = (uint32_t*)(s->ws + L.off_start2);
    s->status = (unsigned long long*)(s->ws + L.off_status);
    s->ticket = (unsigned long long*)(s->ws + L.off_ticket);
    s->tiles[0] = (uint32_t*)(s->ws + L.off_tiles);
    s->tiles[1] = s->tiles[0] + (size_t)sort_blocks((uint32_t)L.ncells) * kTileSpread;
    s->tile_off = (uint32_t*)(s->ws + L.off_toff);
    s->obs_slots = (long long*)(s->ws + L.off_obs);
    s->acc = (double*)(s->ws + L.off_acc);
    s->series = (double*)(s->ws + L.off_series);
    s->dbg_n = (uint32_t*)(s->ws + L.off_dbg_n);
    s->dbg_C = (float*)(s->ws + L.off_dbg_C);
    s->dbg_S = (float*)(s->ws + L.off_dbg_S);
    s->htab = (float*)(s->ws + L.off_h);
    s->hbins = (uint32_t*)(s->ws + L.off_hbins);
    s->hacc = (unsigned long long*)(s->ws + L.off_hacc);
    if (p->weights) s->weights.assign(p->weights, p->weights + p->weight_len);
    s->err = (uint32_t*)(s->ws + L.off_err);
    s->d_step = (uint32_t*)(s->ws + L.off_dstep);
    s->timers.resize(kTCount);
    s->timers[kTScan].name = "k_scan";
    s->timers[kTScatter].name = "k_scatter";
    s->timers[kTNbr].name = "k_nbr";
    s->timers[kTSort].name = "k_sort";

    Geom& g = s->g;
    g.Lxf = (float)p->Lx;
    g.Lyf = (float)p->Ly;
    g.Lx = (double)g.Lxf;
    g.Ly = (double)g.Lyf;
    g.twoLx = 2.0 * g.Lx;
    g.twoLy = 2.0 * g.Ly;
    g.Mx = L.Mx;
    g.My = L.My;
    g.invx = (double)L.Mx / g.Lx;
    g.invy = (double)L.My / g.Ly;
    g.R2 = p->R * p->R;
    g.bx = p->bx ? 1 : 0;
    g.by = p->by ? 1 : 0;
    {
        // cell rows a particle can cross in one step: |dy| is at most the
        // displacement v (VM) or v dt (Langevin) plus the rounding of the
        // binary32 update (relative 2^-20, absolute L 2^-22); re-insertion at
        // a wall or across a periodic edge does not increase it
        const double disp = std::fabs(p->rule != AAP_RULE_LANGEVIN ? p->v : p->v * p->dt);
        const double rows = (disp * (1.0 + 0x1p-20) + g.Ly * 0x1p-22) * ((double)L.My / g.Ly);
        s->rows_per_step = (uint32_t)std::floor(rows) + 1u;
    }
    {
        // Pre-filter bands of the neighbour test (cs = larger cell side,
        // stencil offsets |dx|, |dy| < 2 cs, d2 < 8 cs^2):
        //  - plain pairs: each binary32 difference is the exact difference
        //    times (1 + d), |d| <= 2^-24, and d2 = fma(dx, dx, dy * dy) adds
        //    two more roundings, so |d2f - d2| < 6 * 2^-24 * 8 cs^2 < 2.9e-6 cs^2
        //    (5 * 2^-24 * 8 cs^2 without the fma); band half-width
        //    2^-16 cs^2 = 1.5e-5 cs^2;
        //  - shifted images (x +- L, 2L - x): the image coordinate itself is
        //    rounded, |error| <= 2^-24 (L + 2 cs) per axis, so
        //    |d2f - d2| < 12 * 2^-24 (L + 4 cs) cs; band half-width
        //    2^-19 (L + 4 cs) cs + 2^-16 cs^2 (2.6x that bound).
        const double cs = std::max(g.Lx / g.Mx, g.Ly / g.My);
        const double Lm = std::max(g.Lx, g.Ly);
        prefilter_band(g.R2, 0x1p-16 * cs * cs, s->r2_lo, s->r2_hi);
        prefilter_band(g.R2, 0x1p-19 * (Lm + 4.0 * cs) * cs + 0x1p-16 * cs * cs, s->r2_lo_edge,
                       s->r2_hi_edge);
    }

    Model& m = s->m;
    m.rule = p->rule;
    m.order = p->order;
    if (p->rule != AAP_RULE_LANGEVIN) {
        m.v_step = (float)p->v;
        m.omega_step = (float)p->omega;
        m.eta_pi = (float)(p->eta * M_PI);
        m.gamma_dt = 0.f;
        m.noise_amp = 0.f;
    } else {
        m.v_step = (float)(p->v * p->dt);
        m.omega_step = (float)(p->omega * p->dt);
        m.eta_pi = 0.f;
        m.gamma_dt = (float)(p->gamma * p->dt);
        m.noise_amp = (float)(p->eta * std::sqrt(p->dt));
    }
    m.h = p->weights ? s->htab : nullptr;
    m.hlen = p->weights ? p->weight_len : 0;
    m.key0 = (uint32_t)p->seed;
    m.key1 = (uint32_t)(p->seed >> 32);
    m.replica = p->replica;

    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return fail(AAP_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    }
    {
        // the allocation-free fields entry point's scratch on this device,
        // looked up here so that its calls make no runtime lookup; a failure
        // is reported by that entry point, which tries again
        void* unused = nullptr;
        const std::string keep = g_err;
        if (noalloc_scratch(s->device, &unused) != AAP_OK) g_err = keep;
    }
    rc = [&]() -> int {
        if (p->weights) {
            std::vector<float> h(p->weight_len);
            for (int k = 0; k < p->weight_len; ++k) h[k] = (float)p->weights[k];
            AAP_HIP(hipMemcpyAsync(s->htab, h.data(), h.size() * 4, hipMemcpyHostToDevice,
                                   s->stream));
            AAP_HIP(hipStreamSynchronize(s->stream));
        }
        AAP_HIP(hipMemsetAsync(s->ws + L.off_status, 0, (L.off_acc - L.off_status),
                               s->stream));
        AAP_HIP(hipMemsetAsync(s->acc, 0, 16 * 8, s->stream));
        AAP_HIP(hipMemsetAsync(s->err, 0, 4, s->stream));
        AAP_HIP(launch_init(s->candA, s->oriA, (uint32_t)p->N, g, m.key0, m.key1, m.replica,
                            s->stream));
        return rebuild_cells(s);
    }();
    if (rc) {
        delete s;
        return rc;
    }
    *out = s;
    return AAP_OK;
}

int aap_destroy(aap_sim* s) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    (void)hipStreamSynchronize(s->stream);
    for (auto& t : s->timers)
        for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    sim_drop_graphs(s);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    delete s;
    return AAP_OK;
}

int aap_graph(aap_sim* s, int32_t steps_per_graph) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    if (steps_per_graph < 0 || (steps_per_graph & 1) || steps_per_graph > 4096)
        return fail(AAP_EINVAL, "steps per graph must be 0 or even, at most 4096");
    if (steps_per_graph != s->graph_steps) {
        AAP_HIP(hipStreamSynchronize(s->stream));
        sim_drop_graphs(s);
        s->graph_steps = steps_per_graph;
    }
    return AAP_OK;
}

int aap_step(aap_sim* s, int64_t nsteps, int measure, double* p_series) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(AAP_EINVAL, "nsteps must be >= 0");
    if (p_series && !measure) return fail(AAP_EINVAL, "p_series needs measure != 0");
    if (s->step + (uint64_t)nsteps > 0xFFFFFFFFull)
        return fail(AAP_EINVAL, "step counter would exceed 2^32-1");
    int64_t done = 0;
    while (done < nsteps) {
        const int64_t chunk = p_series ? std::min<int64_t>(nsteps - done, kSeriesCap)
                                       : nsteps - done;
        for (int64_t k = 0; k < chunk;) {
            // a captured run of graph_steps steps, once the state is sorted
            // and the fold of the last measured state is the one the graph
            // starts with (the first measured step of a call is launched)
            if (!p_series && s->graph_steps > 0 && chunk - k >= s->graph_steps && !s->fresh &&
                !s->timing && !s->debug && s->step >= 1 && s->obs_pending == (measure != 0)) {
                hipGraphExec_t e = nullptr;
                const int rc = sim_graph(s, measure != 0, &e);
                if (rc) return rc;
                AAP_HIP(launch_fill_u32(s->d_step, 1, (uint32_t)(s->step - 1), s->stream));
                AAP_HIP(hipGraphLaunch(e, s->stream));
                s->step += (uint64_t)s->graph_steps;
                s->obs_pending = measure != 0;
                s->obs_slot = -1;
                if (s->graph_steps & 1) {
                    s->cur = 1 - s->cur;
                    s->tcur = 1 - s->tcur;
                }
                k += s->graph_steps;
                continue;
            }
            const int rc = one_step(s, measure != 0, p_series != nullptr, (uint32_t)k);
            if (rc) return rc;
            ++k;
        }
        {
            const int rc = finalize_obs(s);
            if (rc) return rc;
        }
        if (p_series) {
            AAP_HIP(hipMemcpyAsync(p_series + done, s->series, (size_t)chunk * 8,
                                   hipMemcpyDeviceToHost, s->stream));
            const int rc = check_device_error(s);
            if (rc) return rc;
        }
        done += chunk;
    }
    return AAP_OK;
}

int aap_sync(aap_sim* s) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    return check_device_error(s);
}

int aap_observables(aap_sim* s, aap_observables_t* out) {
    if (!s || !out) return fail(AAP_EINVAL, "NULL argument");
    int rc = finalize_obs(s);
    if (rc) return rc;
    double acc[16];
    AAP_HIP(hipMemcpyAsync(acc, s->acc, sizeof acc, hipMemcpyDeviceToHost, s->stream));
    rc = check_device_error(s);
    if (rc) return rc;
    std::memset(out, 0, sizeof *out);
    const double n = acc[8];
    out->steps_measured = (int64_t)n;
    if (n > 0) {
        for (int k = 0; k < 4; ++k) {
            out->p_mom[k] = acc[k] / n;
            out->nbar_mom[k] = acc[4 + k] / n;
        }
        const double p2 = out->p_mom[1];
        out->binder = p2 > 0 ? 1.0 - out->p_mom[3] / (3.0 * p2 * p2) : 0.0;
        out->p_last = acc[9];
        out->nbar_last = acc[10];
        for (int k = 0; k < 4; ++k) out->q_mom[k] = acc[11 + k] / n;
        out->q_last = acc[15];
    }
    return AAP_OK;
}

int aap_histograms(aap_sim* s, double* theta_hist, int32_t bins_theta, double* n_hist,
                   int32_t bins_n) {
    if (!s || !theta_hist || !n_hist) return fail(AAP_EINVAL, "NULL argument");
    if (s->p.bins_theta == 0) return fail(AAP_EINVAL, "created without histograms");
    if (bins_theta != s->p.bins_theta || bins_n != s->p.bins_n)
        return fail(AAP_EINVAL, "bin counts differ from the simulation's (%d, %d)",
                    s->p.bins_theta, s->p.bins_n);
    int rc = finalize_obs(s);
    if (rc) return rc;
    const size_t nb = (size_t)(bins_theta + bins_n);
    std::vector<unsigned long long> h(nb);
    double acc8 = 0.0;
    AAP_HIP(hipMemcpyAsync(h.data(), s->hacc, nb * 8, hipMemcpyDeviceToHost, s->stream));
    AAP_HIP(hipMemcpyAsync(&acc8, s->acc + 8, 8, hipMemcpyDeviceToHost, s->stream));
    rc = check_device_error(s);
    if (rc) return rc;
    const double tot = acc8 * (double)s->p.N;   // particles over the measured states
    for (int k = 0; k < bins_theta; ++k) theta_hist[k] = tot > 0 ? (double)h[k] / tot : 0.0;
    for (int k = 0; k < bins_n; ++k) n_hist[k] = tot > 0 ? (double)h[bins_theta + k] / tot : 0.0;
    return AAP_OK;
}

int aap_reset_observables(aap_sim* s) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    const int rc = finalize_obs(s);
    if (rc) return rc;
    AAP_HIP(hipMemsetAsync(s->acc, 0, 16 * 8, s->stream));
    if (s->p.bins_theta > 0)
        AAP_HIP(hipMemsetAsync(s->hacc, 0, (size_t)(s->p.bins_theta + s->p.bins_n) * 8,
                               s->stream));
    return AAP_OK;
}

int aap_get_state(aap_sim* s, float* x, float* y, float* theta, uint64_t* step) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    const size_t N = (size_t)s->p.N;
    std::vector<Cand> c;
    std::vector<Ori> o;
    const int rc = fetch_state(s, c, o);
    if (rc) return rc;
    for (size_t k = 0; k < N; ++k) {
        const uint32_t id = o[k].y;
        if (id >= N) return fail(AAP_EHIP, "corrupt particle id %u", id);
        float xv, yv, tv;
        std::memcpy(&xv, &c[k].x, 4);
        std::memcpy(&yv, &c[k].y, 4);
        std::memcpy(&tv, &o[k].x, 4);
        if (x) x[id] = xv;
        if (y) y[id] = yv;
        if (theta) theta[id] = tv;
    }
    if (step) *step = s->step;
    return AAP_OK;
}

int aap_set_state(aap_sim* s, const float* x, const float* y, const float* theta,
                  uint64_t step) {
    if (!s || !x || !y || !theta) return fail(AAP_EINVAL, "NULL argument");
    if (step > 0xFFFFFFFFull) return fail(AAP_EINVAL, "step must be < 2^32");
    const size_t N = (size_t)s->p.N;
    std::vector<Cand> c;
    std::vector<Ori> o;
    try {
        c.resize(N);
        o.resize(N);
    } catch (...) {
        return fail(AAP_ENOMEM, "host allocation failed");
    }
    const float Lx = s->g.Lxf, Ly = s->g.Lyf;
    for (size_t i = 0; i < N; ++i) {
        const float xi = x[i], yi = y[i], ti = theta[i];
        if (!(std::isfinite(xi) && std::isfinite(yi) && std::isfinite(ti)))
            return fail(AAP_EINVAL, "non-finite state at particle %zu", i);
        const bool okx = s->g.bx ? (xi >= 0.f && xi <= Lx) : (xi >= 0.f && xi < Lx);
        const bool oky = s->g.by ? (yi >= 0.f && yi <= Ly) : (yi >= 0.f && yi < Ly);
        if (!okx || !oky)
            return fail(AAP_EINVAL, "particle %zu outside the box (%g, %g)", i, xi, yi);
        if (!(std::fabs(ti) <= (float)M_PI))
            return fail(AAP_EINVAL, "angle of particle %zu outside [-pi, pi] (%g)", i, ti);
        int32_t xb, yb;
        uint32_t tb;
        std::memcpy(&xb, &xi, 4);
        std::memcpy(&yb, &yi, 4);
        std::memcpy(&tb, &ti, 4);
        c[i] = make_int4(xb, yb, 0, 0);
        o[i] = make_uint2(tb, (uint32_t)i);
    }
    int rc = finalize_obs(s);
    if (rc) return rc;
    AAP_HIP(hipMemcpyAsync(s->candA, c.data(), N * sizeof(Cand), hipMemcpyHostToDevice,
                           s->stream));
    AAP_HIP(hipMemcpyAsync(s->oriA, o.data(), N * sizeof(Ori), hipMemcpyHostToDevice,
                           s->stream));
    rc = rebuild_cells(s);
    if (rc) return rc;
    AAP_HIP(hipStreamSynchronize(s->stream));
    s->step = step;
    s->debug_valid = false;
    return AAP_OK;
}

int aap_debug_keys(aap_sim* s, uint32_t* key, int32_t* mx, int32_t* my) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    if (mx) *mx = s->lay.Mx;
    if (my) *my = s->lay.My;
    if (!key) return AAP_OK;
    const size_t N = (size_t)s->p.N;
    std::vector<Ori> o(N);
    std::vector<uint32_t> k(N);
    AAP_HIP(hipMemcpyAsync(o.data(), s->oriA, N * sizeof(Ori), hipMemcpyDeviceToHost,
                           s->stream));
    AAP_HIP(hipMemcpyAsync(k.data(), s->key, N * 4, hipMemcpyDeviceToHost, s->stream));
    const int rc = check_device_error(s);
    if (rc) return rc;
    for (size_t q = 0; q < N; ++q) {
        const uint32_t id = o[q].y;
        if (id >= N) return fail(AAP_EHIP, "corrupt particle id %u", id);
        key[id] = k[q];
    }
    return AAP_OK;
}

int aap_debug_enable(aap_sim* s, int on) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    s->debug = on != 0;
    s->debug_valid = false;
    return AAP_OK;
}

int aap_debug_last_step(aap_sim* s, uint32_t* start, uint32_t* order, uint32_t* n, float* C,
                        float* S) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    if (!s->debug_valid)
        return fail(AAP_EINVAL, "no step ran with capture enabled since the last change");
    const size_t N = (size_t)s->p.N;
    if (start)
        AAP_HIP(hipMemcpyAsync(start, s->startbuf[s->cur], (s->lay.ncells + 1) * 4,
                               hipMemcpyDeviceToHost, s->stream));
    std::vector<Ori> o(N);
    std::vector<uint32_t> dn(N);
    std::vector<float> dc(N), ds(N);
    AAP_HIP(hipMemcpyAsync(o.data(), s->oriA, N * sizeof(Ori), hipMemcpyDeviceToHost,
                           s->stream));
    AAP_HIP(hipMemcpyAsync(dn.data(), s->dbg_n, N * 4, hipMemcpyDeviceToHost, s->stream));
    AAP_HIP(hipMemcpyAsync(dc.data(), s->dbg_C, N * 4, hipMemcpyDeviceToHost, s->stream));
    AAP_HIP(hipMemcpyAsync(ds.data(), s->dbg_S, N * 4, hipMemcpyDeviceToHost, s->stream));
    const int rc = check_device_error(s);
    if (rc) return rc;
    for (size_t q = 0; q < N; ++q) {
        const uint32_t id = o[q].y;
        if (id >= N) return fail(AAP_EHIP, "corrupt particle id %u", id);
        if (order) order[q] = id;
        if (n) n[id] = dn[q];
        if (C) C[id] = dc[q];
        if (S) S[id] = ds[q];
    }
    return AAP_OK;
}

int aap_timing_enable(aap_sim* s, int every) {
    if (!s) return fail(AAP_EINVAL, "handle is NULL");
    if (every < 0) return fail(AAP_EINVAL, "timing period must be >= 0");
    if (s->timing) {
        const int rc = drain_timers(s);
        if (rc) return rc;
    }
    s->timing = every > 0;
    s->timing_now = false;
    s->timing_every = every;
    s->timing_count = 0;
    for (auto& t : s->timers) {
        t.total_ms = 0.0;
        t.launches = 0;
    }
    return AAP_OK;
}

int aap_timing_read(aap_sim* s, const char** names, double* ms, int64_t* launches,
                    int32_t* count) {
    if (!s || !count) return fail(AAP_EINVAL, "NULL argument");
    const int rc = drain_timers(s);
    if (rc) return rc;
    const int n = std::min<int>(*count, (int)s->timers.size());
    for (int k = 0; k < n; ++k) {
        const TimerSlot& t = s->timers[k];
        if (names) names[k] = t.name;
        if (ms) ms[k] = t.launches ? t.total_ms / (double)t.launches : 0.0;
        if (launches) launches[k] = t.launches;
    }
    *count = (int32_t)s->timers.size();
    return AAP_OK;
}

namespace {

// Checkpoint layout: CkptHeader, weight table (weight_len doubles), x, y,
// theta (N binary32 each, by particle id), the 16 measurement accumulators
// (binary64), the histogram counts (bins_theta + bins_n uint64).
struct CkptHeader {
    char magic[8];
    uint32_t version, header_bytes;
    uint64_t N, step, seed;
    double Lx, Ly, R, v, eta, omega, gamma, dt;
    int32_t rule, order, bx, by, weight_len, bins_theta, bins_n;
    uint32_t replica;
};
constexpr char kCkptMagic[8] = {'A', 'A', 'P', 'C', 'K', 'P', 'T', '1'};

size_t ckpt_size(const aap_sim* s) {
    const size_t N = (size_t)s->p.N;
    return sizeof(CkptHeader) + s->weights.size() * 8 + 3 * N * 4 + 16 * 8 +
           (size_t)(s->p.bins_theta + s->p.bins_n) * 8;
}

CkptHeader ckpt_header(const aap_sim* s) {
    CkptHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = 1;
    h.header_bytes = sizeof h;
    h.N = s->p.N;
    h.step = s->step;
    h.seed = s->p.seed;
    h.Lx = s->g.Lx;
    h.Ly = s->g.Ly;
    h.R = s->p.R;
    h.v = s->p.v;
    h.eta = s->p.eta;
    h.omega = s->p.omega;
    h.gamma = s->p.gamma;
    h.dt = s->p.dt;
    h.rule = s->p.rule;
    h.order = s->p.order;
    h.bx = s->g.bx;
    h.by = s->g.by;
    h.weight_len = (int32_t)s->weights.size();
    h.bins_theta = s->p.bins_theta;
    h.bins_n = s->p.bins_n;
    h.replica = s->p.replica;
    return h;
}

}  // namespace

int aap_checkpoint_bytes(aap_sim* s, size_t* bytes) {
    if (!s || !bytes) return fail(AAP_EINVAL, "NULL argument");
    *bytes = ckpt_size(s);
    return AAP_OK;
}

int aap_checkpoint_save(aap_sim* s, void* buf, size_t bytes) {
    if (!s || !buf) return fail(AAP_EINVAL, "NULL argument");
    if (bytes < ckpt_size(s)) return fail(AAP_EINVAL, "buffer smaller than aap_checkpoint_bytes");
    const size_t N = (size_t)s->p.N;
    unsigned char* o = (unsigned char*)buf;
    const CkptHeader h = ckpt_header(s);
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    if (!s->weights.empty()) {
        std::memcpy(o, s->weights.data(), s->weights.size() * 8);
        o += s->weights.size() * 8;
    }
    float* x = (float*)o;
    float* y = x + N;
    float* t = y + N;
    int rc = aap_get_state(s, x, y, t, nullptr);   // also folds pending measurements
    if (rc) return rc;
    o += 3 * N * 4;
    rc = finalize_obs(s);
    if (rc) return rc;
    AAP_HIP(hipMemcpyAsync(o, s->acc, 16 * 8, hipMemcpyDeviceToHost, s->stream));
    o += 16 * 8;
    const size_t nb = (size_t)(s->p.bins_theta + s->p.bins_n);
    if (nb) AAP_HIP(hipMemcpyAsync(o, s->hacc, nb * 8, hipMemcpyDeviceToHost, s->stream));
    AAP_HIP(hipStreamSynchronize(s->stream));
    return AAP_OK;
}

int aap_checkpoint_load(aap_sim* s, const void* buf, size_t bytes) {
    if (!s || !buf) return fail(AAP_EINVAL, "NULL argument");
    if (bytes < sizeof(CkptHeader)) return fail(AAP_EINVAL, "buffer too small for a checkpoint");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 1 ||
        h.header_bytes != sizeof h)
        return fail(AAP_EINVAL, "not a checkpoint of this library");
    CkptHeader mine = ckpt_header(s);
    mine.step = h.step;
    if (std::memcmp(&mine, &h, sizeof h) != 0)
        return fail(AAP_EINVAL, "checkpoint of a simulation with other parameters");
    if (bytes < ckpt_size(s)) return fail(AAP_EINVAL, "truncated checkpoint");
    const size_t N = (size_t)s->p.N;
    const unsigned char* in = (const unsigned char*)buf + sizeof h;
    if (!s->weights.empty()) {
        if (std::memcmp(in, s->weights.data(), s->weights.size() * 8) != 0)
            return fail(AAP_EINVAL, "checkpoint of a simulation with another weight table");
        in += s->weights.size() * 8;
    }
    const float* x = (const float*)in;
    int rc = aap_set_state(s, x, x + N, x + 2 * N, h.step);
    if (rc) return rc;
    in += 3 * N * 4;
    AAP_HIP(hipMemcpyAsync(s->acc, in, 16 * 8, hipMemcpyHostToDevice, s->stream));
    in += 16 * 8;
    const size_t nb = (size_t)(s->p.bins_theta + s->p.bins_n);
    if (nb) AAP_HIP(hipMemcpyAsync(s->hacc, in, nb * 8, hipMemcpyHostToDevice, s->stream));
    AAP_HIP(hipStreamSynchronize(s->stream));
    return AAP_OK;
}

// ---------------------------------------------------------------------------
// Batches of replicas: independent systems stepped together, each workgroup
// of one launch per kernel working for one replica.
// ---------------------------------------------------------------------------
}  // extern "C"

struct aap_batch {
    std::vector<aap_sim*> reps;
    hipStream_t stream = nullptr;   // the caller's
    hipStream_t cap = nullptr;      // private stream for graph capture
    NbrArgs* nbr_tab = nullptr;     // device: [2][count], by the parity of the sorted state
    SortArgs* sort_tab = nullptr;   // device: [2][count]
    // neighbour workgroups of 64, 128, 256 lanes: replica of each workgroup,
    // first workgroup of each replica, workgroup count
    uint32_t* nbr_b2r[3] = {};
    uint32_t* nbr_b0[3] = {};
    uint32_t nbr_blocks[3] = {};
    int nbr_sel = 2;                // the size in use (index into 64, 128, 256)
    uint32_t* sort_b2r = nullptr;
    uint32_t* sort_b0 = nullptr;
    uint32_t* d_step = nullptr;     // step of the last neighbour launch
    uint32_t sort_blocks_total = 0;
    int rule = 0, bx = 0, by = 0;
    int cur = 0;                    // parity of the current sorted state (all replicas)
    bool fresh = true;              // the next step sorts each replica's given state
    bool prev_meas = false;         // the last step measured (its sums are not folded yet)
    uint64_t step = 0;
    bool debug = false;             // the neighbour tables write n, C, S of every replica
    bool debug_ran = false;         // a step ran since debug output was switched on
    int graph_steps = 0;            // steps per captured graph (0: direct launches)
    hipGraph_t graph[3][2][2] = {};   // [workgroup size][measure][parity at the start]
    hipGraphExec_t exec[3][2][2] = {};
};

namespace {

constexpr int kBatchThreads[3] = {64, 128, 256};

struct BatchLayout {
    size_t off_nbr_tab, off_sort_tab, off_nbr_b2r[3], off_nbr_b0[3], off_sort_b2r, off_sort_b0,
        off_step, off_reps;
    std::vector<size_t> rep_off, rep_bytes;
    uint32_t nbr_blocks[3] = {}, sort_blocks = 0;
    size_t bytes = 0;
};

int batch_layout(const aap_params* params, int32_t count, BatchLayout* out) {
    if (!params) return fail(AAP_EINVAL, "params is NULL");
    if (count < 1 || count > 65536) return fail(AAP_EINVAL, "replica count must be in [1, 65536]");
    BatchLayout L;
    uint64_t nb[3] = {0, 0, 0}, sb = 0;
    for (int32_t r = 0; r < count; ++r) {
        const aap_params* p = params + r;
        Layout lay;
        const int rc = validate(p, &lay);
        if (rc) return fail(rc, "replica %d: %s", r, g_err.c_str());
        if (p->rule != params[0].rule || (p->bx != 0) != (params[0].bx != 0) ||
            (p->by != 0) != (params[0].by != 0))
            return fail(AAP_EINVAL, "replica %d: rule and boundaries must be those of replica 0", r);
        if (p->bins_theta != 0)
            return fail(AAP_EINVAL, "replica %d: histograms are not measured in a batch", r);
        L.rep_bytes.push_back(lay.bytes);
        for (int k = 0; k < 3; ++k) nb[k] += (p->N + kBatchThreads[k] - 1) / kBatchThreads[k];
        sb += sort_blocks((uint32_t)lay.ncells);
    }
    if (nb[0] > 0x7FFFFFFFull || sb > 0x7FFFFFFFull)
        return fail(AAP_EINVAL, "too many workgroups in the batch");
    for (int k = 0; k < 3; ++k) L.nbr_blocks[k] = (uint32_t)nb[k];
    L.sort_blocks = (uint32_t)sb;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.off_nbr_tab = take(2 * (size_t)count * sizeof(NbrArgs));
    L.off_sort_tab = take(2 * (size_t)count * sizeof(SortArgs));
    for (int k = 0; k < 3; ++k) {
        L.off_nbr_b2r[k] = take((size_t)nb[k] * 4);
        L.off_nbr_b0[k] = take((size_t)count * 4);
    }
    L.off_sort_b2r = take((size_t)sb * 4);
    L.off_sort_b0 = take((size_t)count * 4);
    L.off_step = take(4);
    L.off_reps = o;
    for (int32_t r = 0; r < count; ++r) L.rep_off.push_back(take(L.rep_bytes[r]));
    L.bytes = o;
    *out = std::move(L);
    return AAP_OK;
}

void batch_drop_graphs(aap_batch* b) {
    for (auto& size : b->exec)
        for (auto& row : size)
            for (auto& e : row)
                if (e) {
                    (void)hipGraphExecDestroy(e);
                    e = nullptr;
                }
    for (auto& size : b->graph)
        for (auto& row : size)
            for (auto& g : row)
                if (g) {
                    (void)hipGraphDestroy(g);
                    g = nullptr;
                }
}

void batch_free(aap_batch* b) {
    batch_drop_graphs(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (aap_sim* r : b->reps) aap_destroy(r);
    delete b;
}

// The replicas' own bookkeeping after batched steps (they run in lockstep).
void batch_sync_reps(aap_batch* b) {
    for (aap_sim* r : b->reps) {
        r->cur = b->cur;
        r->tcur = b->cur;
        r->step = b->step;
        r->fresh = b->fresh;
        r->obs_pending = b->prev_meas;
        r->obs_slot = -1;
        r->debug_valid = b->debug && b->debug_ran;
    }
}

// The neighbour argument tables of both parities (debug output on or off),
// uploaded synchronously.
int batch_upload_nbr_tables(aap_batch* b) {
    const size_t count = b->reps.size();
    std::vector<NbrArgs> nt(2 * count);
    for (size_t r = 0; r < count; ++r)
        for (int c = 0; c < 2; ++c)
            nt[(size_t)c * count + r] = nbr_args(b->reps[r], c, c, true, false, b->debug);
    AAP_HIP(hipMemcpyAsync(b->nbr_tab, nt.data(), nt.size() * sizeof(NbrArgs),
                           hipMemcpyHostToDevice, b->stream));
    AAP_HIP(hipStreamSynchronize(b->stream));
    return AAP_OK;
}

// The two launches of one sorted step on stream st; fold: the previous step
// measured.  Flips the parity.
int batch_launch_step(aap_batch* b, int& cur, bool fold, bool measure, hipStream_t st,
                      hipEvent_t* ev = nullptr) {
    const size_t R = b->reps.size();
    const int k = b->nbr_sel;
    AAP_HIP(launch_sort_batch(b->sort_tab + (size_t)cur * R, b->sort_b2r, b->sort_b0,
                              b->sort_blocks_total, b->d_step, fold ? 1 : 0, st,
                              ev ? ev[0] : nullptr, ev ? ev[1] : nullptr));
    cur = 1 - cur;
    AAP_HIP(launch_nbr_batch(b->nbr_tab + (size_t)cur * R, b->nbr_b2r[k], b->nbr_b0[k],
                             b->nbr_blocks[k], b->d_step, measure ? 1 : 0, b->rule, b->bx, b->by,
                             kBatchThreads[k], st, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr));
    return AAP_OK;
}

// A graph of graph_steps measured (or unmeasured) steps starting at parity
// cur, captured on the private stream on first use.
int batch_graph(aap_batch* b, bool measure, int cur, hipGraphExec_t* out) {
    hipGraphExec_t& e = b->exec[b->nbr_sel][measure ? 1 : 0][cur];
    if (!e) {
        hipGraph_t& g = b->graph[b->nbr_sel][measure ? 1 : 0][cur];
        AAP_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        int c = cur;
        int rc = AAP_OK;
        for (int k = 0; k < b->graph_steps && rc == AAP_OK; ++k)
            rc = batch_launch_step(b, c, measure, measure, b->cap);
        hipGraph_t got = nullptr;
        const hipError_t ee = hipStreamEndCapture(b->cap, &got);
        if (rc) {
            if (got) (void)hipGraphDestroy(got);
            return rc;
        }
        if (ee != hipSuccess) return fail(AAP_EHIP, "graph capture: %s", hipGetErrorString(ee));
        g = got;
        AAP_HIP(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
    }
    *out = e;
    return AAP_OK;
}

}  // namespace

extern "C" {

int aap_batch_workspace_bytes(const aap_params* params, int32_t count, size_t* bytes) {
    if (!bytes) return fail(AAP_EINVAL, "bytes is NULL");
    BatchLayout L;
    const int rc = batch_layout(params, count, &L);
    if (rc) return rc;
    *bytes = L.bytes;
    return AAP_OK;
}

int aap_batch_create(const aap_params* params, int32_t count, void* d_workspace, size_t bytes,
                     void* hip_stream, aap_batch** out) {
    if (!out) return fail(AAP_EINVAL, "out is NULL");
    *out = nullptr;
    BatchLayout L;
    int rc = batch_layout(params, count, &L);
    if (rc) return rc;
    if (!d_workspace) return fail(AAP_EINVAL, "workspace is NULL");
    if (((uintptr_t)d_workspace & 255) != 0) return fail(AAP_ENOMEM, "workspace not 256-B aligned");
    if (bytes < L.bytes)
        return fail(AAP_ENOMEM, "workspace of %zu B is smaller than the %zu B needed", bytes,
                    L.bytes);
    aap_batch* b = new (std::nothrow) aap_batch;
    if (!b) return fail(AAP_ENOMEM, "host allocation failed");
    unsigned char* ws = (unsigned char*)d_workspace;
    b->stream = (hipStream_t)hip_stream;
    b->rule = params[0].rule;
    b->bx = params[0].bx != 0;
    b->by = params[0].by != 0;
    b->nbr_tab = (NbrArgs*)(ws + L.off_nbr_tab);
    b->sort_tab = (SortArgs*)(ws + L.off_sort_tab);
    for (int k = 0; k < 3; ++k) {
        b->nbr_b2r[k] = (uint32_t*)(ws + L.off_nbr_b2r[k]);
        b->nbr_b0[k] = (uint32_t*)(ws + L.off_nbr_b0[k]);
        b->nbr_blocks[k] = L.nbr_blocks[k];
    }
    b->sort_b2r = (uint32_t*)(ws + L.off_sort_b2r);
    b->sort_b0 = (uint32_t*)(ws + L.off_sort_b0);
    b->d_step = (uint32_t*)(ws + L.off_step);
    b->sort_blocks_total = L.sort_blocks;
    for (int32_t r = 0; r < count; ++r) {
        aap_sim* s = nullptr;
        rc = aap_create(params + r, ws + L.rep_off[r], L.rep_bytes[r], hip_stream, &s);
        if (rc) {
            const std::string msg = g_err;
            batch_free(b);
            return fail(rc, "replica %d: %s", r, msg.c_str());
        }
        b->reps.push_back(s);
    }
    // workgroup tables and the per-replica arguments of both parities
    std::vector<uint32_t> nb2r[3], nb0[3], sb2r, sb0;
    std::vector<NbrArgs> nt(2 * (size_t)count);
    std::vector<SortArgs> st(2 * (size_t)count);
    for (int32_t r = 0; r < count; ++r) {
        const aap_sim* s = b->reps[r];
        for (int k = 0; k < 3; ++k) {
            nb0[k].push_back((uint32_t)nb2r[k].size());
            nb2r[k].insert(nb2r[k].end(), (size_t)((s->p.N + kBatchThreads[k] - 1) / kBatchThreads[k]),
                           (uint32_t)r);
        }
        sb0.push_back((uint32_t)sb2r.size());
        sb2r.insert(sb2r.end(), (size_t)sort_blocks((uint32_t)s->lay.ncells), (uint32_t)r);
        for (int c = 0; c < 2; ++c) {
            nt[(size_t)c * count + r] = nbr_args(s, c, c, true, false, false);
            st[(size_t)c * count + r] = sort_args_of(s, c);
        }
    }
    rc = [&]() -> int {
        AAP_HIP(hipMemcpyAsync(b->nbr_tab, nt.data(), nt.size() * sizeof(NbrArgs),
                               hipMemcpyHostToDevice, b->stream));
        AAP_HIP(hipMemcpyAsync(b->sort_tab, st.data(), st.size() * sizeof(SortArgs),
                               hipMemcpyHostToDevice, b->stream));
        for (int k = 0; k < 3; ++k) {
            AAP_HIP(hipMemcpyAsync(b->nbr_b2r[k], nb2r[k].data(), nb2r[k].size() * 4,
                                   hipMemcpyHostToDevice, b->stream));
            AAP_HIP(hipMemcpyAsync(b->nbr_b0[k], nb0[k].data(), nb0[k].size() * 4,
                                   hipMemcpyHostToDevice, b->stream));
        }
        AAP_HIP(hipMemcpyAsync(b->sort_b2r, sb2r.data(), sb2r.size() * 4, hipMemcpyHostToDevice,
                               b->stream));
        AAP_HIP(hipMemcpyAsync(b->sort_b0, sb0.data(), sb0.size() * 4, hipMemcpyHostToDevice,
                               b->stream));
        AAP_HIP(launch_fill_u32(b->d_step, 1, 0u, b->stream));
        AAP_HIP(hipStreamSynchronize(b->stream));
        AAP_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        return AAP_OK;
    }();
    if (rc) {
        batch_free(b);
        return rc;
    }
    b->cur = b->reps[0]->cur;
    *out = b;
    return AAP_OK;
}

int aap_batch_destroy(aap_batch* b) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    return AAP_OK;
}

int aap_batch_graph(aap_batch* b, int32_t steps_per_graph) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    if (steps_per_graph < 0 || (steps_per_graph & 1) || steps_per_graph > 4096)
        return fail(AAP_EINVAL, "steps per graph must be 0 or even, at most 4096");
    if (steps_per_graph != b->graph_steps) {
        AAP_HIP(hipStreamSynchronize(b->stream));
        batch_drop_graphs(b);
        b->graph_steps = steps_per_graph;
    }
    return AAP_OK;
}

int aap_batch_threads(aap_batch* b, int32_t threads) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    for (int k = 0; k < 3; ++k)
        if (kBatchThreads[k] == threads) {
            b->nbr_sel = k;
            return AAP_OK;
        }
    return fail(AAP_EINVAL, "neighbour workgroup size must be 64, 128 or 256 (got %d)", threads);
}

int aap_batch_kernel_times(aap_batch* b, int32_t steps, int measure, double* sort_ms,
                           double* nbr_ms) {
    if (!b || !sort_ms || !nbr_ms) return fail(AAP_EINVAL, "NULL argument");
    if (steps < 1 || steps > 4096) return fail(AAP_EINVAL, "steps must be in [1, 4096]");
    if (b->step + (uint64_t)steps + 1 > 0xFFFFFFFFull)
        return fail(AAP_EINVAL, "step counter would pass 2^32");
    int rc = AAP_OK;
    if (b->fresh) {
        rc = aap_batch_step(b, 1, measure);
        if (rc) return rc;
    }
    const bool meas = measure != 0;
    if (b->debug) b->debug_ran = true;
    std::vector<hipEvent_t> ev(4 * (size_t)steps, nullptr);
    for (auto& e : ev)
        if (hipEventCreateWithFlags(&e, hipEventDefault) != hipSuccess) {
            rc = fail(AAP_EHIP, "event creation failed");
            break;
        }
    for (int32_t k = 0; k < steps && rc == AAP_OK; ++k) {
        rc = batch_launch_step(b, b->cur, b->prev_meas, meas, b->stream, ev.data() + 4 * k);
        b->prev_meas = meas;
        b->step += 1;
    }
    double ts = 0.0, tn = 0.0;
    if (rc == AAP_OK && hipStreamSynchronize(b->stream) != hipSuccess)
        rc = fail(AAP_EHIP, "stream synchronisation failed");
    for (int32_t k = 0; k < steps && rc == AAP_OK; ++k) {
        float a = 0.f, c = 0.f;
        if (hipEventElapsedTime(&a, ev[4 * k], ev[4 * k + 1]) != hipSuccess ||
            hipEventElapsedTime(&c, ev[4 * k + 2], ev[4 * k + 3]) != hipSuccess) {
            rc = fail(AAP_EHIP, "event timing failed");
            break;
        }
        ts += a;
        tn += c;
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    batch_sync_reps(b);
    if (rc) return rc;
    *sort_ms = ts / steps;
    *nbr_ms = tn / steps;
    return AAP_OK;
}

int aap_batch_autotune(aap_batch* b, int32_t steps, int measure, int32_t* threads,
                       int32_t* steps_per_graph) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    if (steps < 2 || (steps & 1) || steps > 4096)
        return fail(AAP_EINVAL, "trial length must be even, in [2, 4096]");
    int rc = AAP_OK;
    if (b->fresh) {
        rc = aap_batch_step(b, 1, measure);
        if (rc) return rc;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    AAP_HIP(hipEventCreate(&e0));
    AAP_HIP(hipEventCreate(&e1));
    const int graphs[2] = {0, steps};
    float best = 0.f;
    int best_sel = b->nbr_sel, best_graph = b->graph_steps;
    for (int k = 0; k < 3 && rc == AAP_OK; ++k) {
        for (int gi = 0; gi < 2 && rc == AAP_OK; ++gi) {
            b->nbr_sel = k;
            rc = aap_batch_graph(b, graphs[gi]);
            // one untimed trial (captures the graph), one timed
            if (rc == AAP_OK) rc = aap_batch_step(b, steps, measure);
            if (rc == AAP_OK && hipEventRecord(e0, b->stream) != hipSuccess)
                rc = fail(AAP_EHIP, "event record failed");
            if (rc == AAP_OK) rc = aap_batch_step(b, steps, measure);
            if (rc == AAP_OK && hipEventRecord(e1, b->stream) != hipSuccess)
                rc = fail(AAP_EHIP, "event record failed");
            float ms = 0.f;
            if (rc == AAP_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(AAP_EHIP, "event timing failed");
            if (rc == AAP_OK && (best == 0.f || ms < best)) {
                best = ms;
                best_sel = k;
                best_graph = graphs[gi];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    b->nbr_sel = best_sel;
    rc = aap_batch_graph(b, best_graph);
    if (rc) return rc;
    if (threads) *threads = kBatchThreads[best_sel];
    if (steps_per_graph) *steps_per_graph = best_graph;
    return AAP_OK;
}

int aap_batch_step(aap_batch* b, int64_t nsteps, int measure) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(AAP_EINVAL, "nsteps must be >= 0");
    if (b->step + (uint64_t)nsteps > 0xFFFFFFFFull)
        return fail(AAP_EINVAL, "step counter would pass 2^32");
    const bool meas = measure != 0;
    if (nsteps > 0 && b->debug) b->debug_ran = true;
    int64_t k = 0;
    while (k < nsteps) {
        if (b->fresh) {
            // each replica's first step after its initial state: the
            // single-system path, which sorts a state in any order
            for (aap_sim* r : b->reps) {
                const int rc = one_step(r, meas, false, 0);
                if (rc) return rc;
            }
            AAP_HIP(launch_fill_u32(b->d_step, 1, (uint32_t)b->step, b->stream));
            b->fresh = false;
            b->prev_meas = meas;
            b->step += 1;
            k += 1;
            continue;
        }
        if (b->graph_steps > 0 && b->prev_meas == meas && nsteps - k >= b->graph_steps) {
            hipGraphExec_t e = nullptr;
            const int rc = batch_graph(b, meas, b->cur, &e);
            if (rc) return rc;
            AAP_HIP(hipGraphLaunch(e, b->stream));
            b->step += (uint64_t)b->graph_steps;
            k += b->graph_steps;
            continue;
        }
        const int rc = batch_launch_step(b, b->cur, b->prev_meas, meas, b->stream);
        if (rc) return rc;
        b->prev_meas = meas;
        b->step += 1;
        k += 1;
    }
    batch_sync_reps(b);
    return AAP_OK;
}

int aap_batch_sync(aap_batch* b) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    AAP_HIP(hipStreamSynchronize(b->stream));
    for (aap_sim* r : b->reps) {
        const int rc = check_device_error(r);
        if (rc) return rc;
    }
    return AAP_OK;
}

int aap_batch_observables(aap_batch* b, aap_observables_t* out, int32_t count) {
    if (!b || !out) return fail(AAP_EINVAL, "NULL argument");
    if (count != (int32_t)b->reps.size())
        return fail(AAP_EINVAL, "count %d differs from the batch's %zu replicas", count,
                    b->reps.size());
    for (int32_t r = 0; r < count; ++r) {
        const int rc = aap_observables(b->reps[r], out + r);
        if (rc) return rc;
    }
    b->prev_meas = false;   // every replica's last measured state is folded now
    return AAP_OK;
}

int aap_batch_reset_observables(aap_batch* b) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    for (aap_sim* r : b->reps) {
        const int rc = aap_reset_observables(r);
        if (rc) return rc;
    }
    b->prev_meas = false;
    return AAP_OK;
}

int aap_batch_get_state(aap_batch* b, int32_t replica, float* x, float* y, float* theta,
                        uint64_t* step) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    if (replica < 0 || replica >= (int32_t)b->reps.size())
        return fail(AAP_EINVAL, "replica %d out of range", replica);
    return aap_get_state(b->reps[replica], x, y, theta, step);
}

int aap_fields(aap_sim* s, int32_t G, float* d_fields, void* d_scratch, size_t scratch_bytes) {
    if (!s || !d_fields || !d_scratch) return fail(AAP_EINVAL, "NULL argument");
    if (G < 1 || G > 4096) return fail(AAP_EINVAL, "grid side must be in [1, 4096]");
    if (scratch_bytes < fields_scratch_bytes(G))
        return fail(AAP_EINVAL, "scratch of %zu B is smaller than the %zu B needed", scratch_bytes,
                    fields_scratch_bytes(G));
    if (((uintptr_t)d_scratch & 7) != 0) return fail(AAP_EINVAL, "scratch not 8-B aligned");
    if (s->p.rule == AAP_RULE_LANGEVIN && s->p.order != 1)
        return fail(AAP_EINVAL, "fields need the unit vectors of order 1");
    if (s->p.Lx != s->p.Ly) return fail(AAP_EINVAL, "fields need a square box");
    AAP_HIP(launch_fields(s->candA, (uint32_t)s->p.N, s->g.Lx, G, d_scratch, d_fields, s->stream));
    return AAP_OK;
}

int aap_batch_debug_enable(aap_batch* b, int on) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    AAP_HIP(hipStreamSynchronize(b->stream));
    b->debug = on != 0;
    b->debug_ran = false;
    for (aap_sim* r : b->reps) {
        r->debug = b->debug;
        r->debug_valid = false;
    }
    return batch_upload_nbr_tables(b);
}

int aap_batch_debug_keys(aap_batch* b, int32_t replica, uint32_t* key, int32_t* mx, int32_t* my) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    if (replica < 0 || replica >= (int32_t)b->reps.size())
        return fail(AAP_EINVAL, "replica %d out of range", replica);
    return aap_debug_keys(b->reps[replica], key, mx, my);
}

int aap_batch_debug_last_step(aap_batch* b, int32_t replica, uint32_t* start, uint32_t* order,
                              uint32_t* n, float* C, float* S) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    if (replica < 0 || replica >= (int32_t)b->reps.size())
        return fail(AAP_EINVAL, "replica %d out of range", replica);
    return aap_debug_last_step(b->reps[replica], start, order, n, C, S);
}

int aap_fields_noalloc(aap_sim* s, int32_t G, float* d_fields) {
    if (!s || !d_fields) return fail(AAP_EINVAL, "NULL argument");
    if (G < 1 || G > kNoAllocMaxG)
        return fail(AAP_EINVAL, "grid side must be in [1, %d] (the static scratch holds %zu B)",
                    kNoAllocMaxG, kNoAllocScratchBytes);
    if (fields_scratch_bytes(G) > kNoAllocScratchBytes)
        return fail(AAP_EINVAL, "grid side %d needs more scratch than the static %zu B", G,
                    kNoAllocScratchBytes);
    if (s->p.rule == AAP_RULE_LANGEVIN && s->p.order != 1)
        return fail(AAP_EINVAL, "fields need the unit vectors of order 1");
    if (s->p.Lx != s->p.Ly) return fail(AAP_EINVAL, "fields need a square box");
    void* ptr = nullptr;
    const int rc = noalloc_scratch(s->device, &ptr);
    if (rc) return rc;
    AAP_HIP(launch_fields(s->candA, (uint32_t)s->p.N, s->g.Lx, G, ptr, d_fields, s->stream));
    return AAP_OK;
}

int aap_batch_fields(aap_batch* b, int32_t replica, int32_t G, float* d_fields, void* d_scratch,
                     size_t scratch_bytes) {
    if (!b) return fail(AAP_EINVAL, "handle is NULL");
    if (replica < 0 || replica >= (int32_t)b->reps.size())
        return fail(AAP_EINVAL, "replica %d out of range", replica);
    return aap_fields(b->reps[replica], G, d_fields, d_scratch, scratch_bytes);
}

const char* aap_last_error(void) { return g_err.c_str(); }

}  // extern "C"

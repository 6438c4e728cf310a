// Internal interface between the host runtime (aap_api.hip) and the gfx950
// kernels (aap_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aap {

// What a neighbour reads of a particle: binary32 x, y (as int bits) and the
// unit vector (cos theta, sin theta) in fixed point, units of 2^-27 -- for
// the Langevin rule of order o, (cos o theta, sin o theta).
typedef int4 Cand;
// What only the particle itself reads: binary32 theta (bits) and its id.
typedef uint2 Ori;

constexpr int kNbrThreads = 64;      // neighbour kernel workgroup (one wave)
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kSortThreads = 512;   // k_sort workgroup
constexpr int kSortTile = 4 * kSortThreads;   // cells per k_sort workgroup
constexpr int kSortItems = 8;        // source particles per k_sort thread and chunk
constexpr int kTileSpread = 16;      // sub-counters per k_sort tile (spreads the atomics)
// From this many sort tiles on, each tile's offset comes from a small scan
// kernel instead of each tile summing the counts of all tiles before it
// (quadratic in the tile count).
constexpr uint32_t kTileScanMin = 1024;
constexpr int kSeriesCap = 4096;     // p values buffered on device per sync
constexpr int kObsSlots = 256;       // slot groups the measured sums are spread over
constexpr int kObsWords = 8;         // int64 words per group (cos, sin, n, cos 2, sin 2)
constexpr int kHistThreads = 1024;   // histogram kernel workgroup
constexpr int kHistItems = 16;       // particles per histogram thread
constexpr int kHistMaxBins = 4096;   // largest angle / neighbour histogram
constexpr int kScatterItems = 1;     // particles per scatter thread
constexpr int kCandPad = 4;          // spare Cand records after the cell-sorted array
constexpr int kTileIdCap = 160;      // ids of the middle cell row staged with them
constexpr int kMaxOrder = 64;        // largest interaction order o of the Langevin rule

// error bits raised by kernels
constexpr uint32_t kErrScatter = 1u;   // a slot beyond N in the scatter
constexpr uint32_t kErrBounds = 4u;    // a cell range beyond N

// Geometry of the box and the cell grid (binary64 decision arithmetic).
struct Geom {
    double Lx, Ly;           // box sides (already rounded to binary32)
    double twoLx, twoLy;     // 2 L, the mirror line x = L images x -> 2L - x
    double invx, invy;       // cells per unit length, M / L
    double R2;               // R * R
    float Lxf, Lyf;
    int32_t Mx, My;
    int32_t bx, by;
};

// Update-rule constants (binary32 arithmetic).
struct Model {
    int32_t rule;      // 0 VM, 1 Langevin, 2 NVM
    int32_t order;     // o of Eq. (5); 1 for VM and NVM
    float v_step;      // VM: v; Langevin: v dt
    float omega_step;  // VM: omega; Langevin: omega dt
    float eta_pi;      // VM: eta * pi (noise = eta pi (2u - 1))
    float gamma_dt;    // Langevin: Gamma dt
    float noise_amp;   // Langevin: eta sqrt(dt)
    const float* h;    // Langevin weight table (device), or nullptr
    int32_t hlen;
    uint32_t key0, key1;   // generator key = seed
    uint32_t replica;      // counter word 2 of every draw
};

struct NbrArgs {
    const Cand* candB;       // cell-sorted particles (any order inside a cell)
    const Ori* oriB;
    const uint32_t* start;   // cell starts, Mx*My + 1
    Cand* candA;             // out: updated particles in (cell, id) order
    Ori* oriA;
    uint32_t* key_out;       // out: next cell per particle (in the output order)
    uint32_t* tile_count;    // out: arrivals per k_sort tile of the next cells (atomic)
    uint32_t* hist_bins;     // out (measured steps with histograms): angle bin | n bin << 16
    double hist_scale;       // angle bins per radian, bins / (2 pi)
    uint32_t hist_bt, hist_bn;   // bin counts (>= 1 when hist_bins is set)
    long long* obs_slots;    // out: measured sums (cos, sin, n), or nullptr
    uint32_t* dbg_n;         // optional per-position |Omega_i|
    float* dbg_C;            // optional per-position C_i
    float* dbg_S;            // optional per-position S_i
    uint32_t* err;
    Geom g;
    Model m;
    uint32_t N;
    uint32_t step;
    const uint32_t* step_dev;   // the step in device memory (captured steps), or nullptr: step
    // binary32 pre-filter of the neighbour test: certain neighbour below lo,
    // certain non-neighbour above hi; the _edge pair is for shifted images
    float r2_lo, r2_hi, r2_lo_edge, r2_hi_edge;
};

// Arguments of the counting sort of one system (one step).
struct SortArgs {
    const Cand* candA;
    const Ori* oriA;
    const uint32_t* key;
    const uint32_t* start_old;
    uint32_t* start_new;
    Cand* candB;
    Ori* oriB;
    const uint32_t* tile_count;
    uint32_t* tile_clear;
    const uint32_t* tile_offset;   // per tile: arrivals of the tiles before it, or nullptr
    long long* obs_slots;
    double* obs_acc;
    double* series;
    uint32_t* err;
    uint32_t* step_dev;      // when set, tile 0 advances the step the next neighbour kernel reads
    uint32_t nblocks, ncells, N, Mx, My, w, periodic_y;
    int32_t fold, slot;
};

// Launch wrappers (aap_kernels.hip).
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t value, hipStream_t st);
hipError_t launch_init(Cand* cand, Ori* ori, uint32_t N, const Geom& g, uint32_t key0,
                       uint32_t key1, uint32_t replica, hipStream_t st);
// order: the harmonic the unit vectors carry (cos o theta, sin o theta)
hipError_t launch_prepare(Cand* cand, const Ori* ori, uint2* kslot, uint32_t* key,
                          uint32_t* count, uint32_t N, const Geom& g, int order, hipStream_t st);
// w: cell rows a particle can cross in one step (>= 1); tile_count: the
// arrivals per tile counted by the neighbour kernel; tile_clear: the other
// tile-count buffer, cleared for the next neighbour kernel
hipError_t launch_sort(const Cand* candA, const Ori* oriA, const uint32_t* key,
                       const uint32_t* start_old, uint32_t* start_new, Cand* candB, Ori* oriB,
                       uint32_t ncells, uint32_t N, uint32_t Mx, uint32_t My, uint32_t w,
                       int periodic_y, const uint32_t* tile_count, uint32_t* tile_clear,
                       const uint32_t* tile_offset, long long* obs_slots, double* obs_acc,
                       double* series, int fold, int slot, uint32_t* err, uint32_t* step_dev,
                       hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// offset[t] = arrivals counted for the tiles before t (exclusive scan of the
// per-tile sums of the kTileSpread sub-counters); one workgroup
hipError_t launch_tile_offsets(const uint32_t* tile_count, uint32_t nblocks, uint32_t* offset,
                               hipStream_t st);
// e0, e1: optional event pair timing the launch (both or neither).
hipError_t launch_scan(uint32_t* count, uint32_t* start, uint32_t ncells,
                       unsigned long long* status, unsigned long long* ticket,
                       long long* obs_slots, double* obs_acc, double* series, int fold,
                       int slot, uint32_t N, hipStream_t st, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
hipError_t launch_scatter(const Cand* candA, const Ori* oriA, const uint2* kslot,
                          const uint32_t* start, Cand* candB, Ori* oriB, uint32_t N,
                          uint32_t* err, hipStream_t st, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);
hipError_t launch_nbr(const NbrArgs& a, hipStream_t st, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
hipError_t launch_obs(long long* obs_slots, double* obs_acc, double* series, int slot,
                      uint32_t N, hipStream_t st);
// The sort arguments launch_sort builds (fold = 0), for the batch tables.
SortArgs sort_args(const Cand* candA, const Ori* oriA, const uint32_t* key,
                   const uint32_t* start_old, uint32_t* start_new, Cand* candB, Ori* oriB,
                   uint32_t ncells, uint32_t N, uint32_t Mx, uint32_t My, uint32_t w,
                   int periodic_y, const uint32_t* tile_count, uint32_t* tile_clear,
                   long long* obs_slots, double* obs_acc, double* series, int slot,
                   uint32_t* err);
// One launch for every replica of a batch: tab holds each replica's
// arguments, blk2rep the replica of each workgroup, blk0 each replica's
// first workgroup; nblocks the total.  The sort advances *d_step, which the
// neighbour kernel reads as the step.
// threads: workgroup size of the batched neighbour kernel (64, 128 or
// 256; blk2rep, blk0 and nblocks count workgroups of that size).
hipError_t launch_sort_batch(const SortArgs* tab, const uint32_t* blk2rep, const uint32_t* blk0,
                             uint32_t nblocks, uint32_t* d_step, int fold, hipStream_t st,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_nbr_batch(const NbrArgs* tab, const uint32_t* blk2rep, const uint32_t* blk0,
                            uint32_t nblocks, const uint32_t* d_step, int meas, int rule,
                            int bx, int by, int threads, hipStream_t st, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);
hipError_t launch_hist(const uint32_t* bins, uint32_t N, uint32_t bt, uint32_t bn,
                       unsigned long long* acc_t, unsigned long long* acc_n, hipStream_t st);

// The error message of the calling thread (aap_last_error); returns code.
int set_error(int code, const char* msg);

// Fields of a state on a G x G grid (aap_surrogate.hip): scratch holds the
// integer accumulators, fields_scratch_bytes(G) bytes; out [3][G][G].
size_t fields_scratch_bytes(int G);
hipError_t launch_fields(const Cand* cand, uint32_t N, double L, int G, void* scratch,
                         float* out, hipStream_t st);

inline uint32_t scan_blocks(uint32_t ncells) {
    return (ncells + kScanTile - 1) / kScanTile;
}

inline uint32_t sort_blocks(uint32_t ncells) {
    return (ncells + kSortTile - 1) / kSortTile;
}

}  // namespace aap

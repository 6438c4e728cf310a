// gfx950 kernels of one metric Vicsek-class time step.
//
// Per step (Sec. 3.2 of the paper: cell lists rebuilt every step, then a
// 3x3 cell scan; Sec. 2: collision then streaming):
//   k_scan     exclusive prefix sum of the per-cell counts (single pass,
//              decoupled look-back between workgroups); also folds the
//              measured sums of the previous step;
//   k_scatter  moves every particle into its cell's range of the
//              cell-sorted arrays;
//   k_nbr      one thread per particle: neighbour sums of Eq. (6) over the
//              3x3 cells (periodic images or wall mirror images, Sec. 2.4),
//              the update rule (Eqs. (1),(2),(4) or (5)), re-insertion into
//              the box, and the write-back in (cell, id) order together with
//              the next cell id, the next histogram and the next slot.
//
// Particle data: Cand = (x, y, cos theta, sin theta), positions binary32 and
// the unit vector in fixed point (units of 2^-27), the 16 bytes a neighbour
// reads; Ori = (theta, id), the 8 bytes only the particle itself reads.
//
// Decisions that produce integers (cell ids, the neighbour test) are taken
// in binary64 from the binary32 coordinates, with the operation sequence
//   image x  = x_j + s (periodic shift s = -L, 0, +L), -x_j, or 2L - x_j
//   dx = ximg - x_i, dy likewise, d2 = dx*dx + dy*dy, neighbour iff d2 <= R*R
//   cell = min((int)(x * (M / L)), M - 1)
// and no contraction into fused multiply-adds.  Everything else is binary32.

#include "aap_internal.h"

#include <hip/hip_ext.h>

#pragma clang fp contract(off)

namespace aap {

namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.15915494309189533577f;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter
// (id, step, replica, purpose), key = seed.
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;
constexpr uint32_t kWeylB = 0xBB67AE85u;

constexpr uint32_t kPurposeNoiseVM = 0u;
constexpr uint32_t kPurposeNoiseGauss = 1u;
constexpr uint32_t kPurposeInit = 2u;

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pA = (uint64_t)kPhiloxMulA * c.x;   // one 32x32->64 multiply
        const uint64_t pB = (uint64_t)kPhiloxMulB * c.z;
        c = make_uint4((uint32_t)(pB >> 32) ^ c.y ^ k0, (uint32_t)pB,
                       (uint32_t)(pA >> 32) ^ c.w ^ k1, (uint32_t)pA);
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return c;
}

// arg(x + i y) for finite (x, y) != (0, 0), in [-pi, pi].  With
// a = min(|x|, |y|) / max(|x|, |y|) in [0, 1], atan(a) = a P(a^2) where P is
// a degree-7 polynomial fitted to atan(a) / a on [0, 1] by Lawson's
// iteratively reweighted least squares; then atan(1/a) = pi/2 - atan(a),
// the left half plane pi - r, and the sign of y.  The binary32 evaluation
// errs by at most 3.2e-7 rad with an exact quotient; the hardware
// reciprocal (1 ulp) adds at most 2.4e-7 rad.
__device__ __forceinline__ float atan2_poly(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
    const float a = mn * __builtin_amdgcn_rcpf(mx);
    const float s = a * a;
    float p = -0x1.09b708p-8f;
    p = __builtin_fmaf(p, s, 0x1.6632c2p-6f);
    p = __builtin_fmaf(p, s, -0x1.ca07e0p-5f);
    p = __builtin_fmaf(p, s, 0x1.8af180p-4f);
    p = __builtin_fmaf(p, s, -0x1.1cd93ap-3f);
    p = __builtin_fmaf(p, s, 0x1.988170p-3f);
    p = __builtin_fmaf(p, s, -0x1.554c3ap-2f);
    p = __builtin_fmaf(p, s, 0x1.ffffeap-1f);
    float r = a * p;
    r = ay > ax ? 1.57079637f - r : r;
    r = x < 0.0f ? 3.14159274f - r : r;
    return __builtin_copysignf(r, y);
}

// 24 high bits as a binary32 in [0, 1), exact.
__device__ __forceinline__ float u24(uint32_t w) {
    return (float)(w >> 8) * 0x1p-24f;
}

__device__ __forceinline__ float wrap_angle(float th) {
    float w = th - kTwoPi * floorf((th + kPi) * kInvTwoPi);
    if (w >= kPi) w -= kTwoPi;
    if (w < -kPi) w += kTwoPi;
    return w;
}

// sin and cos of an angle with |th| <= 4 (stored angles lie in [-pi, pi)):
// Cody-Waite reduction by pi/2 with pi/2 split into three binary32 parts
// (Cody and Waite, Software Manual for the Elementary Functions, 1980),
// then the Taylor series on |r| <= pi/4, sin to r^9 and cos to r^10 (their
// truncation is below 0.05 ulp), evaluated by Horner's rule with fused
// multiply-adds.  Other arguments take the library routine.
__device__ __forceinline__ void sincos_small(float th, float* sn, float* cs) {
    if (!(fabsf(th) <= 4.0f)) {
        sincosf(th, sn, cs);
        return;
    }
    const float kf = rintf(th * 0.636619772367581343f);   // th / (pi/2), rounded
    float r = __builtin_fmaf(-kf, 0x1.921fb6p+0f, th);     // pi/2 = P1 + P2 + P3
    r = __builtin_fmaf(-kf, -0x1.777a5cp-25f, r);
    r = __builtin_fmaf(-kf, -0x1.ee59dap-50f, r);
    const float s = r * r;
    float ps = __builtin_fmaf(s, 0x1.71de3ap-19f, -0x1.a01a02p-13f);   // 1/9!, -1/7!
    ps = __builtin_fmaf(s, ps, 0x1.111112p-7f);                         // 1/5!
    ps = __builtin_fmaf(s, ps, -0x1.555556p-3f);                        // -1/3!
    const float sr = __builtin_fmaf(r * s, ps, r);
    float pc = __builtin_fmaf(s, -0x1.27e4fcp-22f, 0x1.a01a02p-16f);   // -1/10!, 1/8!
    pc = __builtin_fmaf(s, pc, -0x1.6c16c2p-10f);                       // -1/6!
    pc = __builtin_fmaf(s, pc, 0x1.555556p-5f);                         // 1/4!
    pc = __builtin_fmaf(s, pc, -0.5f);
    const float cr = __builtin_fmaf(s, pc, 1.0f);
    // th = r + q pi/2: (sin, cos) = (sr, cr), (cr, -sr), (-sr, -cr), (-cr, sr)
    const int q = (int)kf & 3;
    const float a = (q & 1) ? cr : sr;
    const float b = (q & 1) ? sr : cr;
    *sn = (q & 2) ? -a : a;
    *cs = ((q + 1) & 2) ? -b : b;
}

__device__ __forceinline__ int cell_of(float x, double inv, int M) {
    const double u = (double)x * inv;
    int c = (u < 0.0) ? 0 : (int)u;
    return c > M - 1 ? M - 1 : c;
}

__device__ __forceinline__ uint32_t cell_key(float x, float y, const Geom& g) {
    const int cx = cell_of(x, g.invx, g.Mx);
    const int cy = cell_of(y, g.invy, g.My);
    return (uint32_t)cy * (uint32_t)g.Mx + (uint32_t)cx;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}


// A 64-bit value moved across lanes by one DPP pattern (both halves).
template <int CTRL>
__device__ __forceinline__ long long dpp_i64(long long x) {
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return (long long)(((uint64_t)hi << 32) | lo);
}

// The five measured sums of a wave in one pass, exact, for the lanes
// (8 q, q = 0..4) that hold them: each term is summed over groups of 8 lanes
// in int32 (|term| <= 2^27), the 40 group sums are moved so that lane
// 8 q + g holds group g of term q, and those are summed in int64 over each
// group of 8 lanes.  One lane per term then holds the wave's total.
__device__ __forceinline__ long long wave_sums5(int32_t (&v)[5], int lane) {
    constexpr int kQuadXor1 = 0xB1;       // quad_perm [1,0,3,2]
    constexpr int kQuadXor2 = 0x4E;       // quad_perm [2,3,0,1]
    constexpr int kRowHalfMirror = 0x141;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        v[q] += __builtin_amdgcn_update_dpp(0, v[q], kQuadXor1, 0xF, 0xF, false);
        v[q] += __builtin_amdgcn_update_dpp(0, v[q], kQuadXor2, 0xF, 0xF, false);
        v[q] += __builtin_amdgcn_update_dpp(0, v[q], kRowHalfMirror, 0xF, 0xF, false);
    }
    const int from = 4 * 8 * (lane & 7);   // byte address of lane 8 (lane % 8)
    int32_t t = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int32_t x = __builtin_amdgcn_ds_bpermute(from, v[q]);
        t = (lane >> 3) == q ? x : t;
    }
    long long T = t;
    T += dpp_i64<kQuadXor1>(T);
    T += dpp_i64<kQuadXor2>(T);
    T += dpp_i64<kRowHalfMirror>(T);
    return T;
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2):
// workgroup b runs on XCD b % 8.  Renumbering them so that every XCD takes
// a contiguous run of the logical blocks (the first nb % 8 XCDs one more
// than the others) keeps a particle's cell neighbourhood, and the records
// the next kernel reads back, in one L2.  The map is a permutation of
// [0, nb).
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t x = b & 7u, q = nb >> 3, r = nb & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// The same dealing with each XCD's workgroups split into kXcdBands pieces
// spread over the box: piece s of XCD x is the logical chunk 8 s + x, the
// chunks laid out in that order.  A dense band of rows then falls on several
// XCDs, not on one (one contiguous run per XCD left the XCDs ending up to
// 11 us apart on banded states).  XCD x receives n_x = q + (x < r)
// workgroups, its piece s the ones of index i (b = 8 i + x) in
// [floor(s n_x / S), floor((s+1) n_x / S)); the map is a permutation of
// [0, nb).  Four pieces measured best of 1, 2, 4, 8 on the 2^20 VM state
// (10^4 steps from the start: -1.3 % per step; after 3 10^4 steps -6 %;
// the NVM at 2^19 -1.5 %).  On larger systems -- the 2^24 uniform control
// (+2.8 %), the clustered 4 2^20 Langevin state (+1.9 %) -- the extra chunk
// edges cost more L2 locality than the balance gains: they keep one run
// per XCD (kXcdSpreadMaxN), and so do small systems (kXcdSpreadMinN; at
// N = 4096 each piece is two waves and the spread cost 3 %).
constexpr uint32_t kXcdBands = 4;
constexpr uint32_t kXcdSpreadMinN = 1u << 16, kXcdSpreadMaxN = 1u << 21;
__device__ __forceinline__ bool xcd_spread(uint32_t N) {
    return N >= kXcdSpreadMinN && N <= kXcdSpreadMaxN;
}
__device__ __forceinline__ uint32_t xcd_block_spread() {
    const uint32_t nb = __builtin_amdgcn_readfirstlane(gridDim.x);
    const uint32_t b = __builtin_amdgcn_readfirstlane(blockIdx.x);
    const uint32_t x = b & 7u, i = b >> 3, q = nb >> 3, r = nb & 7u;
    const uint32_t n = q + (x < r ? 1u : 0u);
    uint32_t sp = 0;   // the piece of block i
#pragma unroll
    for (uint32_t t = 1; t < kXcdBands; ++t) sp += i >= (t * n) / kXcdBands ? 1u : 0u;
    // start of chunk 8 sp + x: the pieces before sp of every XCD (r XCDs of
    // q + 1 blocks, 8 - r of q), then piece sp of the XCDs before x
    const uint32_t b1 = (sp * (q + 1u)) / kXcdBands, e1 = ((sp + 1u) * (q + 1u)) / kXcdBands;
    const uint32_t b0 = (sp * q) / kXcdBands, e0 = ((sp + 1u) * q) / kXcdBands;
    const uint32_t xa = x < r ? x : r;   // XCDs before x with q + 1 blocks
    const uint32_t start = r * b1 + (8u - r) * b0 + xa * (e1 - b1) + (x - xa) * (e0 - b0);
    return start + (i - (sp * n) / kXcdBands);
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ---------------------------------------------------------------------------
// Fixed point of the neighbour and observable sums: unit-vector components
// are rounded once to multiples of 2^-27 (|value| <= 2^27 as int32) and
// summed exactly in integers -- eight terms fit an int32, longer sums go to
// int64 -- so the sums do not depend on the summation order.
// ---------------------------------------------------------------------------
constexpr float kFixScale = 134217728.0f;           // 2^27
constexpr double kFixInv = 1.0 / 134217728.0;

__device__ __forceinline__ int32_t to_fix(float v) { return __float2int_rn(v * kFixScale); }

// The angle o theta of the o-th harmonic, reduced to [-pi, pi]: o theta is
// exact in binary64 (o <= 64, theta binary32), the reduction by the binary64
// 2 pi errs by at most 2^-46, and the result is rounded once to binary32.
__device__ __forceinline__ float harmonic_angle(float th, int o) {
    const double t = (double)o * (double)th;
    const double k = rint(t * 0.15915494309189535);   // 1 / (2 pi)
    return (float)(t - k * 6.283185307179586);
}

// Unit vector a neighbour reads: (cos theta, sin theta), or for the Langevin
// rule of order o the harmonic (cos o theta, sin o theta) (Eq. (5)).
__device__ __forceinline__ void unit_vector(float th, int order, float* sn, float* cs) {
    sincos_small(order == 1 ? th : harmonic_angle(th, order), sn, cs);
}

__device__ __forceinline__ Cand make_cand(float x, float y, float th, int order) {
    float sn, cs;
    unit_vector(th, order, &sn, &cs);
    return make_int4(__float_as_int(x), __float_as_int(y), to_fix(cs), to_fix(sn));
}

// Uniform positions and isotropic orientations (the initial condition of
// the paper's runs, Sec. 5), drawn with purpose INIT at step 0.
__global__ void k_init(Cand* __restrict__ cand, Ori* __restrict__ ori, uint32_t N, Geom g,
                       uint32_t k0, uint32_t k1, uint32_t replica) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint4 w = philox10(make_uint4(i, 0u, replica, kPurposeInit), k0, k1);
    float x = g.Lxf * u24(w.x);
    float y = g.Lyf * u24(w.y);
    const float th = kPi * (2.0f * u24(w.z) - 1.0f);
    if (!g.bx && x >= g.Lxf) x -= g.Lxf;
    if (!g.by && y >= g.Lyf) y -= g.Lyf;
    cand[i] = make_int4(__float_as_int(x), __float_as_int(y), 0, 0);
    ori[i] = make_uint2(__float_as_uint(th), i);
}

// For a state given by positions (cand.x, cand.y) and orientations (ori.x),
// in any order: the unit vector of every particle, its cell (kslot.x and
// key), the per-cell histogram, and the particle's slot in its cell (the
// histogram atomic's return value).  The first step after such a state sorts
// with k_scan and k_scatter; later steps sort with k_sort.
__global__ void k_prepare(Cand* __restrict__ cand, const Ori* __restrict__ ori,
                          uint2* __restrict__ kslot, uint32_t* __restrict__ key,
                          uint32_t* __restrict__ count, uint32_t N, Geom g, int order) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const Cand c = cand[i];
    const float x = __int_as_float(c.x), y = __int_as_float(c.y);
    cand[i] = make_cand(x, y, __uint_as_float(ori[i].x), order);
    const uint32_t k = cell_key(x, y, g);
    kslot[i] = make_uint2(k, atomicAdd(&count[k], 1u));
    key[i] = k;
}

// ---------------------------------------------------------------------------
// Measured observables (Sec. 3.4).  Every neighbour-kernel wave adds its
// fixed-point sums (cos th, sin th, cos 2th, sin 2th in units of 2^-27, and
// n) to one of kObsSlots groups of kObsWords int64 slots with integer
// atomics (order independent).  obs_finalize, run by one wave after that
// kernel, folds the slots into the polar order p = |sum e^{i th}| / N, the
// nematic order q = |sum e^{2i th}| / N and nbar = sum n / N of the
// pre-update state, accumulates their moments k = 1..4 in acc[0..3] (p),
// acc[4..7] (nbar) and acc[11..14] (q), counts the state in acc[8], keeps the
// last p, nbar, q in acc[9], acc[10], acc[15], and clears the slots.
// ---------------------------------------------------------------------------
constexpr double kFixInvObs = 1.0 / 134217728.0;   // 2^-27

__device__ void obs_finalize(long long* slots, double* acc, double* series, int32_t slot,
                             uint32_t N) {
    const int lane = threadIdx.x & 63;
    long long c = 0, s = 0, n = 0, c2 = 0, s2 = 0;
    for (int k = lane; k < kObsSlots; k += 64) {
        long long* w = slots + k * kObsWords;
        c += w[0];
        s += w[1];
        n += w[2];
        c2 += w[3];
        s2 += w[4];
        w[0] = 0;
        w[1] = 0;
        w[2] = 0;
        w[3] = 0;
        w[4] = 0;
    }
    c = wave_sum_i64(c);
    s = wave_sum_i64(s);
    n = wave_sum_i64(n);
    c2 = wave_sum_i64(c2);
    s2 = wave_sum_i64(s2);
    if (lane == 0) {
        const double C = (double)c * kFixInvObs, S = (double)s * kFixInvObs;
        const double C2 = (double)c2 * kFixInvObs, S2 = (double)s2 * kFixInvObs;
        const double p = sqrt(C * C + S * S) / (double)N;
        const double q = sqrt(C2 * C2 + S2 * S2) / (double)N;
        const double nb = (double)n / (double)N;
        double pk = 1.0, nk = 1.0, qk = 1.0;
        for (int k = 0; k < 4; ++k) {
            pk *= p;
            nk *= nb;
            qk *= q;
            acc[k] += pk;
            acc[4 + k] += nk;
            acc[11 + k] += qk;
        }
        acc[8] += 1.0;
        acc[9] = p;
        acc[10] = nb;
        acc[15] = q;
        if (series && slot >= 0) series[slot] = p;
    }
}

__global__ __launch_bounds__(64) void k_obs(long long* slots, double* acc, double* series,
                                            int32_t slot, uint32_t N) {
    obs_finalize(slots, acc, series, slot, N);
}

// ---------------------------------------------------------------------------
// Exclusive scan of the cell counts: one pass, decoupled look-back.
// A 64-bit ticket counter, never reset, hands out block indices in start
// order (so a block only waits on blocks already running) and an epoch
// (launch number) that tags every status word:
//   status[b] = epoch << 34 | flag << 32 | value,
// flag 1 = block aggregate, 2 = inclusive prefix.  Words of older launches
// carry an older epoch and are ignored, so nothing is cleared between
// launches (safe under graph replay).  The block with index 0 also folds the
// observables of the previous (measured) step when asked to (fold != 0),
// last, after its prefix is out.
// ---------------------------------------------------------------------------
constexpr unsigned long long kFlagAgg = 1ull;
constexpr unsigned long long kFlagIncl = 2ull;

__device__ __forceinline__ void status_store(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long status_load(unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long status_word(unsigned long long epoch,
                                                          unsigned long long flag, uint32_t v) {
    return (epoch << 34) | (flag << 32) | (unsigned long long)v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan(
    uint32_t* __restrict__ count, uint32_t* __restrict__ start, uint32_t ncells,
    unsigned long long* status, unsigned long long* ticket, uint32_t nblocks,
    long long* obs_slots, double* obs_acc, double* series, int32_t fold, int32_t slot,
    uint32_t N) {
    __shared__ uint32_t s_bid;
    __shared__ unsigned long long s_epoch;
    __shared__ uint32_t s_wsum[kScanThreads / 64];
    __shared__ uint32_t s_prefix;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        const unsigned long long tk = __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
        s_bid = (uint32_t)(tk % nblocks);
        s_epoch = ((tk / nblocks) + 1ull) & 0x3FFFFFFFull;
    }
    __syncthreads();
    const uint32_t b = s_bid;
    const unsigned long long epoch = s_epoch;
    const uint64_t base = (uint64_t)b * kScanTile + (uint64_t)tid * kScanItems;

    uint32_t v[kScanItems];
    // read the histogram and leave zeros for the next one
    if (base + kScanItems <= ncells) {
        uint4* p4 = reinterpret_cast<uint4*>(count + base);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            const uint4 t = p4[q];
            v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
        }
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) p4[q] = make_uint4(0u, 0u, 0u, 0u);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = (base + k < ncells) ? count[base + k] : 0u;
            if (base + k < ncells) count[base + k] = 0u;
        }
    }
    uint32_t tsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) tsum += v[k];
    const uint32_t incl = wave_incl_scan(tsum, lane);
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, btotal = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        const uint32_t s = s_wsum[w];
        if (w < wave) woff += s;
        btotal += s;
    }
    if (wave == 0) {
        uint32_t prefix = 0;
        if (b == 0) {
            if (lane == 0) status_store(&status[0], status_word(epoch, kFlagIncl, btotal));
        } else {
            if (lane == 0) status_store(&status[b], status_word(epoch, kFlagAgg, btotal));
            int64_t pos = (int64_t)b - 1;
            while (true) {
                const int64_t idx = pos - lane;
                unsigned long long fl = kFlagIncl;   // before block 0: prefix 0
                uint32_t val = 0;
                if (idx >= 0) {
                    unsigned long long st = status_load(&status[idx]);
                    while ((st >> 34) != epoch || ((st >> 32) & 3ull) == 0) {
                        __builtin_amdgcn_s_sleep(1);
                        st = status_load(&status[idx]);
                    }
                    fl = (st >> 32) & 3ull;
                    val = (uint32_t)st;
                }
                const unsigned long long inclmask = __ballot(fl == kFlagIncl);
                const int first = inclmask ? (__ffsll((long long)inclmask) - 1) : 64;
                prefix += wave_sum_u32(lane <= first ? val : 0u);
                if (inclmask) break;
                pos -= 64;
            }
            if (lane == 0)
                status_store(&status[b], status_word(epoch, kFlagIncl, prefix + btotal));
        }
        if (lane == 0) s_prefix = prefix;
    }
    __syncthreads();
    uint32_t run = s_prefix + woff + incl - tsum;
    if (base + kScanItems <= ncells) {
        uint32_t o[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) { o[k] = run; run += v[k]; }
        uint4* q4 = reinterpret_cast<uint4*>(start + base);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q)
            q4[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < ncells) start[base + k] = run;
            run += v[k];
        }
    }
    if (base < ncells && base + kScanItems >= ncells)
        start[ncells] = run;   // thread holding the last cell: total = N
    // after block 0 has published its prefix, so no block waits on the fold
    if (b == 0 && fold && wave == kScanThreads / 64 - 1)
        obs_finalize(obs_slots, obs_acc, series, slot, N);
}

// ---------------------------------------------------------------------------
// Scatter into cell ranges: particle i goes to start[key] + slot, where slot
// is its place in the cell handed out by the histogram atomic when the key
// was computed.  No atomics here; the order inside a cell is arbitrary and
// the neighbour kernel ranks each particle in its cell by id.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter(const Cand* __restrict__ candA,
                                                 const Ori* __restrict__ oriA,
                                                 const uint2* __restrict__ kslot,
                                                 const uint32_t* __restrict__ start,
                                                 Cand* __restrict__ candB, Ori* __restrict__ oriB,
                                                 uint32_t N, uint32_t* err) {
    const uint32_t base = xcd_block() * (256u * kScatterItems) + threadIdx.x;
    uint2 ks[kScatterItems];
    uint32_t st[kScatterItems];
    Cand c[kScatterItems];
    Ori o[kScatterItems];
#pragma unroll
    for (int q = 0; q < kScatterItems; ++q) {
        const uint32_t i = base + (uint32_t)q * 256u;
        ks[q] = make_uint2(0u, 0u);
        if (i < N) {
            ks[q] = kslot[i];
            c[q] = candA[i];
            o[q] = oriA[i];
        }
    }
#pragma unroll
    for (int q = 0; q < kScatterItems; ++q) {
        const uint32_t i = base + (uint32_t)q * 256u;
        st[q] = (i < N) ? start[ks[q].x] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kScatterItems; ++q) {
        const uint32_t i = base + (uint32_t)q * 256u;
        if (i < N) {
            const uint32_t pos = st[q] + ks[q].y;
            if (pos >= N) {
                atomicOr(err, kErrScatter);
            } else {
                candB[pos] = c[q];
                oriB[pos] = o[q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Counting sort of a cell-ordered state into its next cells, one kernel.
// The particles of candA lie in the order of the cells they held (start_old);
// key gives each one's next cell.  A particle crosses at most w cell rows in
// a step, so the particles arriving in a tile of kSortTile cells come from
// the rows of that tile widened by w on each side (cyclically on a periodic
// y axis).  Block b (ticket order, as k_scan):
//   1. counts, with LDS atomics, the particles of those rows whose next cell
//      lies in its tile;
//   2. scans the counts, takes its offset as the number of arrivals in the
//      tiles before it (counted per tile by the neighbour kernel that made
//      the keys, so no block waits for another), and writes the tile's cell
//      starts;
//   3. moves those particles to start + a slot handed out by a second LDS
//      atomic (any order inside a cell: the neighbour kernel ranks by id).
// Block 0 also clears the other tile-count buffer for the next neighbour
// kernel and folds the previous step's measured sums, last.
// ---------------------------------------------------------------------------
// Tile b of the counting sort of system a; fold: the slots hold a measured
// state still to be folded into the accumulators.
// Dense tiles take more than one chunk of sources: the keys of the second
// chunk are loaded with the first (they stay in registers through the scan),
// so its move needs one memory round trip instead of two.  The first
// kStageCap places of a tile's output range are filled in LDS and then
// written out in order, so every store covers whole lines of the cache (the
// per-particle places in HBM are scattered over the cells of the tile); a
// tile of more arrivals writes its places beyond them directly (on small
// grids all of them).  The batched
// sort does not stage: on its small replicas the extra barrier and copy pass
// cost more than the whole-line stores save (measured: +2 %).
constexpr int kKeptChunks = 1;
constexpr uint32_t kStageCap = 2944;   // arrivals a tile can stage in LDS (2944 x 24 B)
// Partial staging of tiles over kStageCap pays on grids of more tiles than
// the 256 CUs (511 tiles, two per CU: -2 us per sort); on a grid of 128
// tiles, each alone on its CU, the extra copy pass costs +1 us.
constexpr uint32_t kPartialStageTiles = 256;
// Source positions and next cells (relative to the tile at lo) of the
// sources q = c0 + tid + u kSortThreads of one chunk, 0xFFFFFFFF past the
// last source.  Every key load is issued before the first is used: a lane
// past the last source loads the last key instead of branching around its
// load (a load inside a branch with its use would wait there, one round trip
// per load).
__device__ __forceinline__ void chunk_keys(const SortArgs& a, uint32_t c0, int tid, uint32_t p0,
                                           uint32_t n0, uint32_t p2, uint32_t ntot, uint32_t lo,
                                           uint32_t (&src)[kSortItems],
                                           uint32_t (&d)[kSortItems]) {
    uint32_t kv[kSortItems];
#pragma unroll
    for (int u = 0; u < kSortItems; ++u) {
        const uint32_t q = c0 + (uint32_t)tid + (uint32_t)u * kSortThreads;
        src[u] = q < n0 ? p0 + q : p2 + (q - n0);
        kv[u] = a.key[min(src[u], a.N - 1u)];
    }
#pragma unroll
    for (int u = 0; u < kSortItems; ++u) {
        const uint32_t q = c0 + (uint32_t)tid + (uint32_t)u * kSortThreads;
        d[u] = q < ntot ? kv[u] - lo : 0xFFFFFFFFu;
    }
}

// Workgroup barrier for data exchanged through LDS only: waits for the
// wave's LDS operations, not for its global loads and stores, so that loads
// whose results are used after the barrier stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <bool kStage>
__device__ __forceinline__ void sort_tile(const SortArgs& a, uint32_t b, int32_t fold) {
    __shared__ __align__(16) uint32_t h[kSortTile];
    __shared__ Cand s_cand[kStage ? kStageCap : 1];
    __shared__ Ori s_ori[kStage ? kStageCap : 1];
    __shared__ uint32_t s_wsum[kSortThreads / 64];
    __shared__ uint32_t s_part[kSortThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    reinterpret_cast<uint4*>(h)[tid] = make_uint4(0u, 0u, 0u, 0u);   // four cells per thread
    // the tile's offset: arrivals of the tiles before it, as counted by the
    // neighbour kernel (summed here while the histogram is built, four
    // sub-counters per load)
    static_assert(kSortTile == 4 * kSortThreads && kTileSpread % 4 == 0, "16-byte accesses");
    // this tile's own arrival count (the check after the scan), loaded now
    const uint32_t own_part = (tid < 64 && lane < kTileSpread)
                                  ? a.tile_count[b * kTileSpread + (uint32_t)lane] : 0u;
    // the bounds of the source rows first: their loads, the head of the
    // chain to the keys, go out with the tile-count loads below
    const uint32_t lo = b * (uint32_t)kSortTile;
    const uint32_t span = min((uint32_t)kSortTile, a.ncells - lo);
    // source rows [r0, r1] (and [r2, r3] when the window wraps)
    const int rF = (int)(lo / a.Mx), rL = (int)((lo + span - 1u) / a.Mx);
    const int My = (int)a.My, w = (int)a.w;
    int r0 = rF - w, r1 = rL + w, r2 = 0, r3 = -1;
    if (r1 - r0 + 1 >= My) {
        r0 = 0;
        r1 = My - 1;
    } else if (a.periodic_y) {
        if (r0 < 0) {
            r2 = r0 + My;
            r3 = My - 1;
            r0 = 0;
        } else if (r1 >= My) {
            r2 = 0;
            r3 = r1 - My;
            r1 = My - 1;
        }
    } else {
        r0 = max(r0, 0);
        r1 = min(r1, My - 1);
    }
    const uint32_t p0 = a.start_old[(uint32_t)r0 * a.Mx];
    const uint32_t p1 = a.start_old[(uint32_t)(r1 + 1) * a.Mx];
    const uint32_t p2 = r3 >= r2 ? a.start_old[(uint32_t)r2 * a.Mx] : 0u;
    const uint32_t p3 = r3 >= r2 ? a.start_old[(uint32_t)(r3 + 1) * a.Mx] : 0u;
    uint32_t before = 0;
    if (a.tile_offset)
        before = tid == 0 ? a.tile_offset[b] : 0u;
    else
        for (uint32_t t = (uint32_t)tid; t < b * (kTileSpread / 4); t += kSortThreads) {
            const uint4 c4 = reinterpret_cast<const uint4*>(a.tile_count)[t];
            before += c4.x + c4.y + c4.z + c4.w;
        }
    if (b == 0)
        for (uint32_t t = (uint32_t)tid; t < a.nblocks * kTileSpread; t += kSortThreads)
            a.tile_clear[t] = 0u;
    lds_barrier();
    const uint32_t n0 = p1 - p0, ntot = n0 + (p3 - p2);
    constexpr uint32_t kChunk = (uint32_t)kSortThreads * kSortItems;

    // 1. histogram of the arrivals, in chunks of kSortItems sources per
    // thread with all their loads in flight; the first chunk's keys and
    // arrival records stay in registers through the scan
    static_assert(kKeptChunks == 1, "one kept chunk");
    uint32_t src[kSortItems], dd[kSortItems];
    uint32_t de[kSortItems];   // next cells of the kept chunk
    Cand cr[kSortItems];
    Ori orr[kSortItems];
    chunk_keys(a, 0u, tid, p0, n0, p2, ntot, lo, src, dd);
    if (kChunk < ntot) {
        uint32_t unused[kSortItems];
        chunk_keys(a, kChunk, tid, p0, n0, p2, ntot, lo, unused, de);
    } else {
#pragma unroll
        for (int u = 0; u < kSortItems; ++u) de[u] = 0xFFFFFFFFu;
    }
#pragma unroll
    for (int u = 0; u < kSortItems; ++u) {
        cr[u] = make_int4(0, 0, 0, 0);
        orr[u] = make_uint2(0u, 0u);
        if (dd[u] < span) {
            atomicAdd(&h[dd[u]], 1u);
            cr[u] = a.candA[src[u]];
            orr[u] = a.oriA[src[u]];
        }
    }
#pragma unroll
    for (int u = 0; u < kSortItems * kKeptChunks; ++u)
        if (de[u] < span) atomicAdd(&h[de[u]], 1u);
    for (uint32_t c0 = (1 + kKeptChunks) * kChunk; c0 < ntot; c0 += kChunk) {
        uint32_t d2[kSortItems], unused[kSortItems];
        chunk_keys(a, c0, tid, p0, n0, p2, ntot, lo, unused, d2);
#pragma unroll
        for (int u = 0; u < kSortItems; ++u)
            if (d2[u] < span) atomicAdd(&h[d2[u]], 1u);
    }
    lds_barrier();

    // 2. block scan (kSortTile / kSortThreads cells per thread), look-back,
    // cell starts
    static_assert(kSortTile == 4 * kSortThreads, "four cells per thread");
    uint4 v = reinterpret_cast<uint4*>(h)[tid];
    const uint32_t tsum = v.x + v.y + v.z + v.w;
    const uint32_t incl = wave_incl_scan(tsum, lane);
    if (lane == 63) s_wsum[wave] = incl;
    lds_barrier();
    uint32_t woff = 0, btotal = 0;
#pragma unroll
    for (int q = 0; q < kSortThreads / 64; ++q) {
        const uint32_t t = s_wsum[q];
        if (q < wave) woff += t;
        btotal += t;
    }
    const uint32_t bpart = wave_sum_u32(before);
    if (lane == 0) s_part[wave] = bpart;
    lds_barrier();
    uint32_t base = 0;
#pragma unroll
    for (int q = 0; q < kSortThreads / 64; ++q) base += s_part[q];
    if (wave == 0) {
        const uint32_t mine = wave_sum_u32(own_part);
        if (lane == 0 && mine != btotal) atomicOr(a.err, kErrScatter);   // counts disagree
    }
    {
        const uint32_t run = woff + incl - tsum;
        const uint4 o = make_uint4(run, run + v.x, run + v.x + v.y, run + v.x + v.y + v.z);
        reinterpret_cast<uint4*>(h)[tid] = o;   // exclusive offsets, the cursors of step 3
        const uint32_t c0 = 4u * (uint32_t)tid;
        if (c0 + 0 < span) a.start_new[lo + c0 + 0] = base + o.x;
        if (c0 + 1 < span) a.start_new[lo + c0 + 1] = base + o.y;
        if (c0 + 2 < span) a.start_new[lo + c0 + 2] = base + o.z;
        if (c0 + 3 < span) a.start_new[lo + c0 + 3] = base + o.w;
        if (lo + span == a.ncells && tid == 0) {
            a.start_new[a.ncells] = base + btotal;
            if (base + btotal != a.N) atomicOr(a.err, kErrScatter);   // a particle went unsorted
        }
    }
    lds_barrier();

    // 3. move the arrivals: the first chunk from registers, the kept chunk
    // with its keys from registers, later chunks re-read with their loads in
    // flight.  The first scap places of the tile's output range are filled in
    // LDS and written out in whole lines afterwards, the places beyond them
    // directly: scap = kStageCap, except for a tile of more arrivals on a
    // grid of fewer than kPartialStageTiles tiles, which writes all directly.
    const uint32_t scap =
        (btotal <= kStageCap || a.nblocks >= kPartialStageTiles) ? kStageCap : 0u;
#pragma unroll
    for (int u = 0; u < kSortItems; ++u) {
        if (dd[u] < span) {
            const uint32_t li = atomicAdd(&h[dd[u]], 1u);
            if (kStage && li < scap) {
                s_cand[li] = cr[u];
                s_ori[li] = orr[u];
            } else if (base + li < a.N) {
                a.candB[base + li] = cr[u];
                a.oriB[base + li] = orr[u];
            } else {
                atomicOr(a.err, kErrScatter);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kKeptChunks; ++k) {
        if ((1u + (uint32_t)k) * kChunk >= ntot) break;
#pragma unroll
        for (int u = 0; u < kSortItems; ++u) {
            const uint32_t q =
                (1u + (uint32_t)k) * kChunk + (uint32_t)tid + (uint32_t)u * kSortThreads;
            src[u] = q < n0 ? p0 + q : p2 + (q - n0);
            dd[u] = de[k * kSortItems + u];
            if (dd[u] < span) {
                cr[u] = a.candA[src[u]];
                orr[u] = a.oriA[src[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < kSortItems; ++u) {
            if (dd[u] < span) {
                const uint32_t li = atomicAdd(&h[dd[u]], 1u);
                if (kStage && li < scap) {
                    s_cand[li] = cr[u];
                    s_ori[li] = orr[u];
                } else if (base + li < a.N) {
                    a.candB[base + li] = cr[u];
                    a.oriB[base + li] = orr[u];
                } else {
                    atomicOr(a.err, kErrScatter);
                }
            }
        }
    }
    for (uint32_t c0 = (1 + kKeptChunks) * kChunk; c0 < ntot; c0 += kChunk) {
        chunk_keys(a, c0, tid, p0, n0, p2, ntot, lo, src, dd);
#pragma unroll
        for (int u = 0; u < kSortItems; ++u) {
            if (dd[u] < span) {
                cr[u] = a.candA[src[u]];
                orr[u] = a.oriA[src[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < kSortItems; ++u) {
            if (dd[u] < span) {
                const uint32_t li = atomicAdd(&h[dd[u]], 1u);
                if (kStage && li < scap) {
                    s_cand[li] = cr[u];
                    s_ori[li] = orr[u];
                } else if (base + li < a.N) {
                    a.candB[base + li] = cr[u];
                    a.oriB[base + li] = orr[u];
                } else {
                    atomicOr(a.err, kErrScatter);
                }
            }
        }
    }
    if (kStage && scap != 0u) {
        lds_barrier();
        for (uint32_t i = (uint32_t)tid; i < min(btotal, scap); i += kSortThreads) {
            if (base + i < a.N) {
                a.candB[base + i] = s_cand[i];
                a.oriB[base + i] = s_ori[i];
            } else {
                atomicOr(a.err, kErrScatter);
            }
        }
    }
    if (b == 0 && fold && wave == kSortThreads / 64 - 1)
        obs_finalize(a.obs_slots, a.obs_acc, a.series, a.slot, a.N);
    if (b == 0 && tid == 0 && a.step_dev) *a.step_dev = *a.step_dev + 1u;
}

// Offsets of the sort tiles for large grids: thread i of one workgroup sums
// the sub-counters of a contiguous range of tiles, the workgroup scans those
// sums, and each thread writes the running offsets of its range.
__global__ __launch_bounds__(1024) void k_tile_offsets(const uint32_t* __restrict__ cnt,
                                                       uint32_t nb, uint32_t* __restrict__ off) {
    __shared__ uint32_t s_w[16];
    const uint32_t tid = threadIdx.x;
    const int lane = (int)(tid & 63u), wave = (int)(tid >> 6);
    const uint32_t per = (nb + 1023u) / 1024u;
    const uint32_t t0 = min(tid * per, nb), t1 = min(t0 + per, nb);
    // a tile's sixteen sub-counters are 64 aligned bytes: four 16-byte loads
    static_assert(kTileSpread == 16, "four 16-byte loads per tile");
    auto tile_sum = [&](uint32_t t) {
        const uint4* c4 = reinterpret_cast<const uint4*>(cnt + (size_t)t * kTileSpread);
        uint32_t s4 = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint4 v = c4[k];
            s4 += v.x + v.y + v.z + v.w;
        }
        return s4;
    };
    uint32_t sum = 0;
    for (uint32_t t = t0; t < t1; ++t) sum += tile_sum(t);
    const uint32_t incl = wave_incl_scan(sum, lane);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int q = 0; q < wave; ++q) run += s_w[q];
    for (uint32_t t = t0; t < t1; ++t) {
        off[t] = run;
        run += tile_sum(t);
    }
}

// Tiles are dealt to the XCDs like the neighbour kernel's blocks (four
// pieces per XCD spread over the box for kXcdSpreadMinN to kXcdSpreadMaxN
// particles, else one run): a tile's rows were written by the neighbour
// kernel on the same XCD, and the rows it shares with its neighbouring tiles
// are read within one L2.
__global__ __launch_bounds__(kSortThreads) void k_sort(SortArgs a) {
    sort_tile<true>(a, __builtin_amdgcn_readfirstlane(
                           xcd_spread(a.N) ? xcd_block_spread() : xcd_block()),
                    a.fold);
}

// Batched form: workgroup gb sorts tile gb - blk0[r] of replica r =
// blk2rep[gb] (round-robin over the XCDs, as in the batched neighbour
// kernel).  Workgroup 0 advances the device step counter that the batched
// neighbour kernel of this step reads.
__global__ __launch_bounds__(kSortThreads) void k_sort_b(const SortArgs* __restrict__ tab,
                                                        const uint32_t* __restrict__ blk2rep,
                                                        const uint32_t* __restrict__ blk0,
                                                        uint32_t* d_step, int32_t fold) {
    const uint32_t gb = blockIdx.x;
    const uint32_t r = blk2rep[gb];
    if (gb == 0 && threadIdx.x == 0) *d_step = *d_step + 1u;
    sort_tile<false>(tab[r], gb - blk0[r], fold);
}

// ---------------------------------------------------------------------------
// Neighbour sums + update + streaming, one thread per particle in cell
// order.  The candidates of a particle in cell (cx, cy) are the particles of
// the 3x3 cells around it.  Away from the box edges these are three
// contiguous ranges of the cell-sorted arrays; in the edge cells the
// neighbouring cells are wrapped (periodic images, shifted by +-L) or
// mirrored (reflecting walls, x -> -x or 2L - x with theta -> pi - theta,
// y likewise with theta -> -theta), Sec. 2.4.  Candidates are read directly
// from the cell-sorted arrays; neighbouring threads share them through the
// L1/L2 caches.
//
// Neighbour test.  The binary64 predicate d2 <= R^2 is decided first in
// binary32: below r2_lo the pair is certainly a neighbour, above r2_hi it
// certainly is not (bands derived from the rounding of the binary32
// differences, wider for shifted images); in between the exact binary64
// sequence decides.  Every decision therefore equals the binary64 one.
//
// Self.  The particle itself is in its own candidate list (d2 = 0) and is
// counted there: it is the e^{i theta_i} term of Eq. (2); n = hits - 1.  Its
// own mirror images next to a reflecting wall are not neighbours (Eq. (6),
// j != i): those that pass the test are taken out afterwards.
// ---------------------------------------------------------------------------
constexpr int kUnroll = 4;   // candidates in flight per thread (4 * 2^27 fits int32)
constexpr int kEdgeUnroll = 4;
constexpr int kImgId = 0, kImgMinusL = 1, kImgPlusL = 2, kImgMirror0 = 3, kImgMirrorL = 4;

__device__ __forceinline__ void map_axis(int v, int M, int refl, int& gidx, int& code) {
    if (v < 0) {
        if (refl) { gidx = 0; code = kImgMirror0; }
        else { gidx = M - 1; code = kImgMinusL; }
    } else if (v >= M) {
        if (refl) { gidx = M - 1; code = kImgMirrorL; }
        else { gidx = 0; code = kImgPlusL; }
    } else {
        gidx = v; code = kImgId;
    }
}

// The image maps of Sec. 2.4 as x -> s x + o: identity (1, 0), periodic
// shifts (1, -L) and (1, +L), mirrors at 0 (-1, 0) and at L (-1, 2L).  s x is
// exact, so s x + o is the one rounding of x - L, x + L, -x or 2L - x.
__device__ __forceinline__ void image_map(int code, float L, float& s, float& o) {
    s = (code >= kImgMirror0) ? -1.0f : 1.0f;
    o = (code == kImgMinusL) ? -L : (code == kImgPlusL) ? L : (code == kImgMirrorL) ? 2.0f * L : 0.0f;
}

// The canonical binary64 neighbour test of an image of j seen from i.
__device__ __forceinline__ bool exact_hit(float xj, float yj, double xi, double yi, double R2) {
    const double dx = (double)xj - xi;
    const double dy = (double)yj - yi;
    const double d2 = dx * dx + dy * dy;
    return d2 <= R2;
}

__device__ __forceinline__ bool exact_hit_map(float xj, float yj, float sx, float ox, float sy,
                                              float oy, double xi, double yi, double R2) {
    const double dx = ((double)sx * (double)xj + (double)ox) - xi;
    const double dy = ((double)sy * (double)yj + (double)oy) - yi;
    const double d2 = dx * dx + dy * dy;
    return d2 <= R2;
}

// Nematic Vicsek rule (Eq. (3)).  A neighbour enters turned by pi when
// cos(th_i - th~_j) < 0 (sign(0) = +1), th~_j its orientation as seen through
// the image map: th_j, pi - th_j (x mirror), -th_j (y mirror), th_j - pi
// (both).
//
// Exact test.  cos(th_i - th~_j) = sigma cos(s) with s = th_i + th_j when
// exactly one mirror applies and th_i - th_j otherwise, sigma = -1 for an x
// mirror.  s is formed in binary64, which is exact for binary32 angles of
// magnitude >= 2^-28; a smaller angle moves s by at most 2^-51 while every
// binary32 number is at least 4.3e-8 from pi/2, so s stays on the same side
// of the zeros of cos.  For |s| <= 2 pi, cos(s) > 0 exactly when |s| < pi/2
// or |s| > 3 pi/2; the two constants are the binary64 numbers next to pi/2
// (below) and 3 pi/2 (above), so both comparisons are exact, and cos(s) = 0
// cannot happen for a binary64 s != 0.
__device__ __forceinline__ bool nvm_aligned(float thi, float thj, bool mx, bool my) {
    const double s = (mx != my) ? (double)thi + (double)thj : (double)thi - (double)thj;
    const double as = fabs(s);
    const bool cos_pos = as <= 0x1.921fb54442d18p+0 || as >= 0x1.2d97c7f3321d3p+2;
    return mx ? !cos_pos : cos_pos;
}

// Fast test.  The dot product of the two stored unit vectors (each component
// within 2^-21 of the exact value) computed in binary32 from the 2^-27 fixed
// point lies within 1.6e-6 * 2^54 of cos(th_i - th~_j) * 2^54; outside the
// band |d| <= 2^-17 * 2^54 its sign is the exact sign, inside it the exact
// test above decides from the angles.
constexpr float kNvmBand = 0x1p37f;

struct OwnVec {
    float c, s;   // the particle's unit vector, units of 2^-27
    float th;     // and its binary32 angle
};

// Turns the (image-mapped) neighbour vector (cz, cw) by pi when the pair is
// anti-aligned.  j: the neighbour's position in the cell-sorted arrays,
// read only when the band is hit (live pairs only).
__device__ __forceinline__ void nvm_orient(int32_t& cz, int32_t& cw, const OwnVec& o, bool mx,
                                           bool my, bool live, uint32_t j, const NbrArgs& a) {
    const float d = __builtin_fmaf(o.c, (float)cz, o.s * (float)cw);
    bool anti = d < 0.0f;
    if (live && !(fabsf(d) > kNvmBand))
        anti = !nvm_aligned(o.th, __uint_as_float(a.oriB[j].x), mx, my);
    cz = anti ? -cz : cz;
    cw = anti ? -cw : cw;
}

struct Acc {
    long long sc, ss, sn;   // fixed-point sums of cos, sin (2^-27) and n
    long long sc2, ss2;     // fixed-point cos 2th, sin 2th
};

// The update rule for one particle given its neighbour sums, the
// re-insertion into the box, and the write-back in (cell, id) order.
template <int RULE, int BX, int BY>
__device__ __forceinline__ void finish_particle(const NbrArgs& a, float xs, float ys,
                                                float thi, int32_t ci_fix, int32_t si_fix,
                                                uint32_t idi, uint32_t n, long long Cf,
                                                long long Sf, uint32_t gpos, uint32_t step,
                                                bool meas, Acc& acc) {
    const Geom& g = a.g;
    // the particle's own unit vector (cos th, sin th); for the Langevin rule
    // of order o >= 2 the stored vector is the o-th harmonic
    int32_t c1_fix = ci_fix, s1_fix = si_fix;
    if (RULE == 1 && a.m.order != 1) {
        float s1, c1;
        sincos_small(thi, &s1, &c1);
        c1_fix = to_fix(c1);
        s1_fix = to_fix(s1);
    }
    acc.sc += c1_fix;
    acc.ss += s1_fix;
    acc.sn += (long long)n;
    if (meas) {
        // e^{2i th} = (c^2 - s^2, 2 c s) from the unit vector
        const double cd = (double)c1_fix * kFixInv, sd = (double)s1_fix * kFixInv;
        acc.sc2 += __double2int_rn((cd * cd - sd * sd) * 134217728.0);
        acc.ss2 += __double2int_rn((2.0 * cd * sd) * 134217728.0);
    }
    // C, S = the sums rounded once to binary32: int32 -> binary32 rounds to
    // nearest like the binary64 path, and the 2^-27 scaling is exact
    float C, S;
    if (__all(Cf == (long long)(int32_t)Cf && Sf == (long long)(int32_t)Sf)) {
        C = (float)(int32_t)Cf * 0x1p-27f;
        S = (float)(int32_t)Sf * 0x1p-27f;
    } else {
        C = (float)((double)Cf * kFixInv);
        S = (float)((double)Sf * kFixInv);
    }
    float x = xs, y = ys, tn, sn = 0.f, cs = 0.f, t_sc = 0.f;
    bool have_sc = false;
    const uint32_t t = step;
    if (RULE != 1) {
        // Vicsek (C, S: the bracket of Eq. (2), or of Eq. (3) for the NVM):
        // arg of the summed unit vectors, chirality, uniform noise
        const float f0 = (Cf == 0 && Sf == 0) ? thi : atan2_poly(S, C);
        const uint4 wv =
            philox10(make_uint4(idi, t, a.m.replica, kPurposeNoiseVM), a.m.key0, a.m.key1);
        const float xi_n = 2.0f * u24(wv.x) - 1.0f;    // exact
        tn = wrap_angle(f0 + a.m.omega_step + a.m.eta_pi * xi_n);
        sincos_small(tn, &sn, &cs);
        t_sc = tn;
        have_sc = true;
        x = x + a.m.v_step * cs;
        y = y + a.m.v_step * sn;
    } else {
        // Langevin (Euler-Maruyama): sum sin(o (th_j - th_i)) =
        // S cos o th_i - C sin o th_i with the o-th harmonic sums C, S
        const float ci = (float)ci_fix * 0x1p-27f;
        const float si = (float)si_fix * 0x1p-27f;
        const float A = ci * S - si * C;
        float hw = 1.0f;
        if (a.m.hlen > 0) {
            const uint32_t k = n < (uint32_t)(a.m.hlen - 1) ? n : (uint32_t)(a.m.hlen - 1);
            hw = a.m.h[k];
        }
        const uint4 wv =
            philox10(make_uint4(idi, t, a.m.replica, kPurposeNoiseGauss), a.m.key0, a.m.key1);
        const float u1 = ((float)(wv.x >> 8) + 1.0f) * 0x1p-24f;   // (0, 1]
        const float u2 = u24(wv.y);
        const float gz = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
        tn = thi + (a.m.gamma_dt * hw * A + a.m.omega_step) + a.m.noise_amp * gz;
        x = x + a.m.v_step * ((float)c1_fix * 0x1p-27f);
        y = y + a.m.v_step * ((float)s1_fix * 0x1p-27f);
    }
    // re-insertion into the box (Sec. 2.4)
    if (BX) {
        if (x < 0.0f) { x = -x; tn = kPi - tn; }
        else if (x > g.Lxf) { x = 2.0f * g.Lxf - x; tn = kPi - tn; }
    } else {
        if (x < 0.0f) x += g.Lxf;
        if (x >= g.Lxf) x -= g.Lxf;
    }
    if (BY) {
        if (y < 0.0f) { y = -y; tn = -tn; }
        else if (y > g.Lyf) { y = 2.0f * g.Lyf - y; tn = -tn; }
    } else {
        if (y < 0.0f) y += g.Lyf;
        if (y >= g.Lyf) y -= g.Lyf;
    }
    tn = wrap_angle(tn);
    // unit vector of the stored orientation, for the next step's sums
    if (RULE == 1 && a.m.order != 1) unit_vector(tn, a.m.order, &sn, &cs);
    else if (!have_sc || tn != t_sc) sincos_small(tn, &sn, &cs);
    if (gpos < a.N) {
        const uint32_t k2 = cell_key(x, y, g);
        a.candA[gpos] = make_int4(__float_as_int(x), __float_as_int(y), to_fix(cs), to_fix(sn));
        a.oriA[gpos] = make_uint2(__float_as_uint(tn), idi);
        a.key_out[gpos] = k2;
        if (a.hist_bins) {
            // histogram bins of the measured state (angle bin decided in
            // binary64 from the binary32 angle; n saturates in the last bin)
            const double u = ((double)thi + 3.14159265358979311600) * a.hist_scale;
            const uint32_t bt = u > 0.0 ? (u < (double)a.hist_bt ? (uint32_t)u : a.hist_bt - 1u)
                                        : 0u;
            const uint32_t bn = n < a.hist_bn - 1u ? n : a.hist_bn - 1u;
            a.hist_bins[gpos] = bt | (bn << 16);
        }
        // arrivals per k_sort tile, one atomic per tile present in the wave,
        // into one of kTileSpread sub-counters chosen by the wave
        const uint32_t t2 = k2 / (uint32_t)kSortTile;
        const uint32_t sub = ((blockIdx.x * (kNbrThreads / 64)) + (threadIdx.x >> 6)) % kTileSpread;
        unsigned long long pending = __ballot(1);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const uint32_t lt = __builtin_amdgcn_readlane(t2, leader);
            const unsigned long long grp = __ballot(t2 == lt) & pending;
            if ((threadIdx.x & 63) == leader)
                atomicAdd(&a.tile_count[lt * kTileSpread + sub], (uint32_t)__popcll(grp));
            pending &= ~grp;
        }
        if (a.dbg_n) {
            a.dbg_n[gpos] = n;
            a.dbg_C[gpos] = C;
            a.dbg_S[gpos] = S;
        }
    } else {
        atomicOr(a.err, kErrBounds);
    }
}

// LDS of one wave: the candidates of its three cell rows, each row followed
// by kUnroll - 1 sentinel records (NaN position: never a neighbour), and
// the ids of its middle row.  The tile holds 280 records (5.1 KB with the
// ids: 32 one-wave workgroups fit a CU's LDS, so the register count, not the
// LDS, sets the occupancy), 320 for the NVM, whose register count allows
// fewer waves anyway and whose clustered states fill larger tiles.
constexpr int tile_cap(int rule) { return rule == 2 ? 320 : 280; }
template <int CAP>
struct WaveLds {
    Cand tile[CAP];
    uint32_t ids[kTileIdCap];
};

// The neighbours among kUnroll candidates of a particle at (xs, ys), the
// first nvalid of which count (all of them without CHECK): fixed-point sums of the batch (exact in
// int32: |term| <= 2^27) and the number of hits.  The binary32 pre-filter
// settles every pair outside the band [r2_lo, r2_hi]; pairs inside it take
// the exact binary64 test in one rarely taken branch per batch.  d2 uses one
// fused multiply-add; its error stays far inside the band.
//
// NVM: each neighbour's vector is oriented by Eq. (3) first (jv: the
// candidates' positions in the cell-sorted arrays, own: the particle's
// vector and angle); the other rules ignore both.
template <bool CHECK, bool NVM>
__device__ __forceinline__ void add_batch(const Cand (&Qv)[kUnroll], uint32_t nvalid, float xs,
                                          float ys, const NbrArgs& a, const OwnVec& own,
                                          const uint32_t (&jv)[kUnroll], int32_t& bc,
                                          int32_t& bs, uint32_t& bn) {
    bool band = false;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const float dx = __int_as_float(Qv[u].x) - xs;
        const float dy = __int_as_float(Qv[u].y) - ys;
        const float d2 = __builtin_fmaf(dx, dx, dy * dy);
        const bool valid = !CHECK || (uint32_t)u < nvalid;
        const bool in = valid & (d2 < a.r2_lo);
        // in the band: d2 <= r2_hi but not below r2_lo (r2_lo < r2_hi)
        band |= valid & ((d2 <= a.r2_hi) != (d2 < a.r2_lo));
        int32_t cz = Qv[u].z, cw = Qv[u].w;
        if (NVM) nvm_orient(cz, cw, own, false, false, in, jv[u], a);
        bc += in ? cz : 0;
        bs += in ? cw : 0;
        bn += in ? 1u : 0u;
    }
    if (band) {
        const double xd = (double)xs, yd = (double)ys;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const float xj = __int_as_float(Qv[u].x), yj = __int_as_float(Qv[u].y);
            const float dx = xj - xs, dy = yj - ys;
            const float d2 = __builtin_fmaf(dx, dx, dy * dy);
            if ((!CHECK || (uint32_t)u < nvalid) && !(d2 < a.r2_lo) && d2 <= a.r2_hi &&
                exact_hit(xj, yj, xd, yd, a.g.R2)) {
                int32_t cz = Qv[u].z, cw = Qv[u].w;
                if (NVM) nvm_orient(cz, cw, own, false, false, true, jv[u], a);
                bc += cz;
                bs += cw;
                bn += 1u;
            }
        }
    }
}

// add_batch for candidates seen through periodic shifts of the axes
// (x -> x + ox, y -> y + oy; each shift 0 or +-L): a shifted coordinate is
// rounded once, so the pre-filter takes the band of shifted images and the
// band's pairs the binary64 test of the image map.  The first nvalid
// candidates count.
template <bool NVM>
__device__ __forceinline__ void add_batch_shift(const Cand (&Qv)[kUnroll], uint32_t nvalid, float xs,
                                                float ys, float ox, float oy, const NbrArgs& a,
                                                const OwnVec& own, const uint32_t (&jv)[kUnroll],
                                                int32_t& bc, int32_t& bs, uint32_t& bn) {
    bool band = false;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const float dx = (__int_as_float(Qv[u].x) + ox) - xs;
        const float dy = (__int_as_float(Qv[u].y) + oy) - ys;
        const float d2 = __builtin_fmaf(dx, dx, dy * dy);
        const bool valid = (uint32_t)u < nvalid;
        const bool in = valid & (d2 < a.r2_lo_edge);
        band |= valid & ((d2 <= a.r2_hi_edge) != (d2 < a.r2_lo_edge));
        int32_t cz = Qv[u].z, cw = Qv[u].w;
        if (NVM) nvm_orient(cz, cw, own, false, false, in, jv[u], a);
        bc += in ? cz : 0;
        bs += in ? cw : 0;
        bn += in ? 1u : 0u;
    }
    if (band) {
        const double xd = (double)xs, yd = (double)ys;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const float xj = __int_as_float(Qv[u].x), yj = __int_as_float(Qv[u].y);
            const float dx = (xj + ox) - xs, dy = (yj + oy) - ys;
            const float d2 = __builtin_fmaf(dx, dx, dy * dy);
            if ((uint32_t)u < nvalid && !(d2 < a.r2_lo_edge) && d2 <= a.r2_hi_edge &&
                exact_hit_map(xj, yj, 1.0f, ox, 1.0f, oy, xd, yd, a.g.R2)) {
                int32_t cz = Qv[u].z, cw = Qv[u].w;
                if (NVM) nvm_orient(cz, cw, own, false, false, true, jv[u], a);
                bc += cz;
                bs += cw;
                bn += 1u;
            }
        }
    }
}

// Rank by id among the particles of [o0, o1) (the own cell), read from the
// cell-sorted ids, four loads in flight per iteration.
__device__ __forceinline__ uint32_t rank_in_cell(const NbrArgs& a, uint32_t o0, uint32_t o1,
                                                 uint32_t idi) {
    uint32_t rank = 0;
    for (uint32_t j = o0; j < o1; j += 4) {
        uint32_t ids[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ids[u] = a.oriB[min(j + (uint32_t)u, o1 - 1u)].y;
#pragma unroll
        for (int u = 0; u < 4; ++u) rank += (j + (uint32_t)u < o1 && ids[u] < idi) ? 1u : 0u;
    }
    return rank;
}

// Rank by id inside the own cell for a wave that has not staged its middle
// row's ids: the ids of the wave's own cells (from lane 0's cell start to
// lane 63's cell end, every lane's cell in between) staged in the wave's tile
// space, free at this point, when they fit it; else read from the
// cell-sorted array.  The caller's next wave barrier orders these LDS reads
// before the tile is written again.
template <int CAP>
__device__ __forceinline__ uint32_t rank_staged(const NbrArgs& a, WaveLds<CAP>& L, uint32_t o0,
                                                uint32_t o1, uint32_t idi, int lane) {
    const uint32_t oA = __builtin_amdgcn_readfirstlane(o0);
    const uint32_t oB = __builtin_amdgcn_readlane(o1, 63);
    const uint32_t m = oB - oA;
    if (m > 4u * (uint32_t)CAP) return rank_in_cell(a, o0, o1, idi);
    uint32_t* ids = reinterpret_cast<uint32_t*>(L.tile);
    for (uint32_t e = (uint32_t)lane; e < m; e += 256u) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = e + 64u * (uint32_t)u;
            v[u] = i < m ? a.oriB[oA + i].y : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = e + 64u * (uint32_t)u;
            if (i < m) ids[i] = v[u];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t rank = 0;
    const uint32_t r0 = o0 - oA, r1 = o1 - oA;
    for (uint32_t e = r0; e < r1; e += 4) {
        uint32_t iv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) iv[u] = ids[min(e + (uint32_t)u, r1 - 1u)];
#pragma unroll
        for (int u = 0; u < 4; ++u) rank += (e + (uint32_t)u < r1 && iv[u] < idi) ? 1u : 0u;
    }
    return rank;
}

// Waves of the wrapped-tile path (wave-uniform; 0 for the other waves that
// hold a lane in an edge cell):
//  1, a seam wave of a periodic x axis: its lanes in two consecutive rows
//     r, r + 1 with 1 <= r and r + 1 <= My - 2, the first lane past column 0
//     and the last before column Mx - 1 (the only x-edge lanes are then at
//     the end of row r and the start of row r + 1);
//  2, a one-row wave whose edge lanes lie at periodic edges only: column 0
//     or Mx - 1 on a periodic x axis (then in rows 2 .. My - 3, where each
//     lane's 16-byte load of four cell starts stays inside the array), row 0
//     or My - 1 on a periodic y axis (Mx, My >= 3: the cells and rows it
//     reads are distinct).
template <int BX, int BY>
__device__ __forceinline__ int wrap_tile(const NbrArgs& a, int cx, int cy) {
    if (BX && BY) return 0;   // every edge is a wall
    const int cyA = __builtin_amdgcn_readfirstlane(cy), cyB = __builtin_amdgcn_readlane(cy, 63);
    const int cxA = __builtin_amdgcn_readfirstlane(cx), cxB = __builtin_amdgcn_readlane(cx, 63);
    const bool x_in = cxA >= 1 && cxB <= a.g.Mx - 2;
    if (!BX && x_in && cyB == cyA + 1 && cyA >= 1 && cyB <= a.g.My - 2) return 1;
    if (cyA == cyB && (x_in ? (!BY || (cyA >= 1 && cyA <= a.g.My - 2))
                            : (!BX && cyA >= 2 && cyA <= a.g.My - 3)))
        return 2;
    return 0;
}

__device__ __forceinline__ uint32_t sel3(int k, uint32_t v0, uint32_t v1, uint32_t v2) {
    return k == 0 ? v0 : (k == 1 ? v1 : v2);
}

// One particle per lane; every lane of the wave calls this (live == false
// for lanes past N, which hold a copy of the last particle, add no work and
// store nothing), so wave-level scans see all 64 lanes.
template <int RULE, int BX, int BY>
__device__ __forceinline__ void nbr_particle(const NbrArgs& a, uint32_t p, bool live, uint32_t step,
                                             bool meas, WaveLds<tile_cap(RULE)>& L, Acc& acc) {
    const Geom& g = a.g;
    const int lane = threadIdx.x & 63;
    // Raised issue priority while the wave sends out its chain of dependent
    // loads (own record, cell starts, candidate tile): on a SIMD shared with
    // waves in their arithmetic loops these requests then leave without
    // waiting for issue slots, and their latency overlaps the others' work.
    // Back to normal once the tile is in LDS (or before the other paths'
    // loops).
    __builtin_amdgcn_s_setprio(2);
    const Cand P = a.candB[p];
    const Ori O = a.oriB[p];
    const float xs = __int_as_float(P.x), ys = __int_as_float(P.y);
    const uint32_t idi = O.y;
    constexpr bool kNvm = RULE == 2;
    constexpr int kCap = tile_cap(RULE);
    const OwnVec me{(float)P.z, (float)P.w, __uint_as_float(O.x)};
    const int cx = cell_of(xs, g.invx, g.Mx), cy = cell_of(ys, g.invy, g.My);
    const uint32_t own = (uint32_t)cy * (uint32_t)g.Mx + (uint32_t)cx;
    uint32_t o0, o1;   // the own cell's bounds in the sorted arrays
    uint32_t rank = 0;   // place by id in the own cell: the output position is o0 + rank
    long long Cf = 0, Sf = 0;
    uint32_t n = 0;
    const bool edge = cx < 1 || cx > g.Mx - 2 || cy < 1 || cy > g.My - 2;
    if (!__any(edge)) {
        // three rows of three cells, each a contiguous window
        const uint32_t r0 = own - (uint32_t)g.Mx - 1u;
        uint32_t a0, a1, b0, b1, c0, c1;
        if constexpr (!kNvm) {
            // the four starts of each row's cells cx-1 .. cx+2 in one 16-byte
            // load (4-byte aligned); the middle row's also bound the own cell
            uint4 sa, sb, sc;
            __builtin_memcpy(&sa, a.start + r0, 16);
            __builtin_memcpy(&sb, a.start + r0 + g.Mx, 16);
            __builtin_memcpy(&sc, a.start + r0 + 2 * g.Mx, 16);
            a0 = sa.x;
            a1 = sa.w;
            b0 = sb.x;
            b1 = sb.w;
            c0 = sc.x;
            c1 = sc.w;
            o0 = sb.y;
            o1 = sb.z;
        } else {
            // the NVM kernel keeps single-word loads (the wide ones did not
            // speed it up)
            a0 = a.start[r0];
            a1 = a.start[r0 + 3];
            b0 = a.start[r0 + g.Mx];
            b1 = a.start[r0 + g.Mx + 3];
            c0 = a.start[r0 + 2 * g.Mx];
            c1 = a.start[r0 + 2 * g.Mx + 3];
            o0 = a.start[own];
            o1 = a.start[own + 1];
        }
        const uint32_t la = a1 - a0, lb = b1 - b0, lc = c1 - c0;
        // Wave tile.  When the wave's particles lie in one cell row (cells
        // cxA..cxB of row cy), the candidates of all its lanes are three
        // contiguous ranges: cells cxA-1..cxB+1 of rows cy-1, cy, cy+1.  The
        // wave copies them once into LDS with coalesced loads, each range
        // followed by kUnroll - 1 sentinels; each lane then walks its three
        // windows there, row by row, in batches of kUnroll.  A batch may run
        // past the lane's window: into cells beyond cx+1 of the same row,
        // more than R away in x (the pre-filter or the binary64 test rejects
        // them), or into the sentinels.  The ids of the middle row come along
        // for the rank.
        const int cyA = __builtin_amdgcn_readfirstlane(cy), cyB = __builtin_amdgcn_readlane(cy, 63);
        const int cxA = __builtin_amdgcn_readfirstlane(cx), cxB = __builtin_amdgcn_readlane(cx, 63);
        bool tiled = false, by_rows = false;
        uint32_t rs0 = 0, rs1 = 0, rs2 = 0, T0 = 0, T1 = 0, T2 = 0;
        if (cyA == cyB) {
            // the six segment bounds (start and end of each row's cells
            // cxA-1 .. cxB+1) in one load by lanes 0..5
            const uint32_t rowA = (uint32_t)(cyA - 1) * (uint32_t)g.Mx;
            const uint32_t lo0 = rowA + (uint32_t)cxA - 1u, hi0 = rowA + (uint32_t)cxB + 2u;
            const uint32_t bi = lane < 3 ? lo0 + (uint32_t)lane * (uint32_t)g.Mx
                                         : hi0 + (uint32_t)(lane - 3) * (uint32_t)g.Mx;
            const uint32_t bv = lane < 6 ? a.start[bi] : 0u;
            rs0 = __builtin_amdgcn_readlane(bv, 0);
            rs1 = __builtin_amdgcn_readlane(bv, 1);
            rs2 = __builtin_amdgcn_readlane(bv, 2);
            T0 = __builtin_amdgcn_readlane(bv, 3) - rs0;
            T1 = __builtin_amdgcn_readlane(bv, 4) - rs1;
            T2 = __builtin_amdgcn_readlane(bv, 5) - rs2;
            tiled = T0 + T1 + T2 + 3 * (kUnroll - 1) <= (uint32_t)kCap &&
                    T1 <= (uint32_t)kTileIdCap;
            by_rows = !tiled;
        }
        if (tiled) {
            constexpr uint32_t kGap = kUnroll - 1;
            const uint32_t s1 = T0 + kGap, s2 = s1 + T1 + kGap, T = s2 + T2 + kGap;
            // every load of the tile and of the ids in flight at once, then
            // the LDS stores
            constexpr int kTileIters = (kCap + 63) / 64;
            constexpr int kIdIters = (kTileIdCap + 63) / 64;
            Cand v[kTileIters];
            uint32_t idv[kIdIters];
#pragma unroll
            for (int k = 0; k < kTileIters; ++k) {
                const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                const bool in0 = e < T0, in1 = e >= s1 && e < s1 + T1, in2 = e >= s2 && e < s2 + T2;
                const uint32_t j = in0 ? rs0 + e : in1 ? rs1 + (e - s1) : rs2 + (e - s2);
                v[k] = make_int4(0x7FC00000, 0x7FC00000, 0, 0);
                if (in0 || in1 || in2) v[k] = a.candB[j];
            }
#pragma unroll
            for (int k = 0; k < kIdIters; ++k) {
                const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                idv[k] = e < T1 ? a.oriB[rs1 + e].y : 0u;
            }
#pragma unroll
            for (int k = 0; k < kTileIters; ++k) {
                const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                if (e < T) L.tile[e] = v[k];
            }
#pragma unroll
            for (int k = 0; k < kIdIters; ++k) {
                const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                if (e < T1) L.ids[e] = idv[k];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            __builtin_amdgcn_s_setprio(0);
            // rank: four LDS reads in flight per iteration (indices clamped
            // to the own cell)
            const uint32_t r0 = o0 - rs1, r1 = o1 - rs1;
            for (uint32_t e = r0; e < r1; e += 4) {
                uint32_t iv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) iv[u] = L.ids[min(e + (uint32_t)u, r1 - 1u)];
#pragma unroll
                for (int u = 0; u < 4; ++u) rank += (e + (uint32_t)u < r1 && iv[u] < idi) ? 1u : 0u;
            }
            const uint32_t wbase[3] = {a0 - rs0, b0 - rs1 + s1, c0 - rs2 + s2};
            const uint32_t wlen[3] = {la, lb, lc};
            const uint32_t wpos[3] = {a0, b0, c0};   // window starts in the sorted arrays
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const Cand* w = L.tile + wbase[r];
                for (uint32_t q = 0; q < wlen[r]; q += kUnroll) {
                    Cand Qv[kUnroll];
                    uint32_t jv[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        Qv[u] = w[q + u];
                        jv[u] = wpos[r] + q + (uint32_t)u;
                    }
                    int32_t bc = 0, bs = 0;
                    uint32_t bn = 0;
                    add_batch<false, kNvm>(Qv, kUnroll, xs, ys, a, me, jv, bc, bs, bn);
                    Cf += bc;
                    Sf += bs;
                    n += bn;
                }
            }
        } else if (by_rows) {
            // Dense waves: the three rows do not fit the tile together.  The
            // rows are staged one after the other into the same LDS tile, a
            // row longer than the tile in pieces of kCap - (kUnroll - 1)
            // records, each row or piece followed by kUnroll - 1 sentinels;
            // each lane walks the part of its window of the row inside the
            // piece, as above.  The rank reads the middle row's ids from LDS
            // when they fit, else from the cell-sorted array.
            constexpr uint32_t kGap = kUnroll - 1;
            constexpr int kTileIters = (kCap + 63) / 64;
            constexpr int kIdIters = (kTileIdCap + 63) / 64;
            if (T1 <= (uint32_t)kTileIdCap) {
#pragma unroll
                for (int k = 0; k < kIdIters; ++k) {
                    const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                    if (e < T1) L.ids[e] = a.oriB[rs1 + e].y;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const uint32_t r0 = o0 - rs1, r1 = o1 - rs1;
                for (uint32_t e = r0; e < r1; e += 4) {
                    uint32_t iv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) iv[u] = L.ids[min(e + (uint32_t)u, r1 - 1u)];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        rank += (e + (uint32_t)u < r1 && iv[u] < idi) ? 1u : 0u;
                }
            } else {
                rank = rank_staged(a, L, o0, o1, idi, lane);
            }
            constexpr uint32_t kPiece = (uint32_t)kCap - kGap;
#pragma unroll 1
            for (int r = 0; r < 3; ++r) {
                const uint32_t Tr = sel3(r, T0, T1, T2), rs = sel3(r, rs0, rs1, rs2);
                const uint32_t ws = sel3(r, a0, b0, c0);
                const uint32_t we = ws + sel3(r, la, lb, lc);   // the lane's window [ws, we)
                for (uint32_t pb = 0; pb < Tr; pb += kPiece) {
                    const uint32_t len = min(kPiece, Tr - pb), g0 = rs + pb;
                    Cand v[kTileIters];
#pragma unroll
                    for (int k = 0; k < kTileIters; ++k) {
                        const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                        v[k] = make_int4(0x7FC00000, 0x7FC00000, 0, 0);
                        if (e < len) v[k] = a.candB[g0 + e];
                    }
                    // every lane is done with the previous piece before it is overwritten
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                    for (int k = 0; k < kTileIters; ++k) {
                        const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                        if (e < len + kGap) L.tile[e] = v[k];
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    // the part of the window in this piece: [lo, hi)
                    const uint32_t lo = max(ws, g0), hi = min(we, g0 + len);
                    const Cand* w = L.tile + (lo - g0);
                    for (uint32_t q = 0; lo + q < hi; q += kUnroll) {
                        Cand Qv[kUnroll];
                        uint32_t jv[kUnroll];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u) {
                            Qv[u] = w[q + u];
                            jv[u] = lo + q + (uint32_t)u;
                        }
                        int32_t bc = 0, bs = 0;
                        uint32_t bn = 0;
                        add_batch<false, kNvm>(Qv, kUnroll, xs, ys, a, me, jv, bc, bs, bn);
                        Cf += bc;
                        Sf += bs;
                        n += bn;
                    }
                }
            }
        } else {
            // the wave spans two cell rows: each lane reads its three
            // windows from the cell-sorted array
            rank = rank_staged(a, L, o0, o1, idi, lane);
            const uint32_t lab = la + lb, tot = lab + lc;
            for (uint32_t q = 0; q < tot; q += kUnroll) {
                Cand Qv[kUnroll];
                uint32_t jv[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const uint32_t qq = min(q + (uint32_t)u, tot - 1u);
                    jv[u] = qq < la ? a0 + qq : (qq < lab ? b0 + (qq - la) : c0 + (qq - lab));
                    Qv[u] = a.candB[jv[u]];
                }
                __builtin_amdgcn_sched_barrier(0);
                int32_t bc = 0, bs = 0;
                uint32_t bn = 0;
                add_batch<true, kNvm>(Qv, tot - q, xs, ys, a, me, jv, bc, bs, bn);
                Cf += bc;
                Sf += bs;
                n += bn;
            }
        }
        n -= 1;   // the particle itself
    } else if (const int wm = wrap_tile<BX, BY>(a, cx, cy); wm != 0) {
        // Wrapped-tile wave.  For each row offset dy the wave's candidates
        // in the rows at dy are one contiguous range of the cell-sorted array
        // (segment dy): for a one-row wave cells cxA-1 .. cxB+1 of row r+dy,
        // within the row; for a seam wave cell cxA-1 of row r+dy through cell
        // cxB+1 of row r+1+dy.  Besides, a lane in column Mx-1 needs cell 0
        // of its row at dy seen at x + L, a lane in column 0 cell Mx-1 of its
        // row at dy seen at x - L (six one-cell segments).  A row across the
        // y edge is seen at y -+ L.  The wave stages the nine segments in
        // LDS, each non-empty one followed by kUnroll - 1 sentinels; a dense
        // wave stages the three range segments only and reads the one-cell
        // segments from the cell-sorted array.  Every lane walks its window
        // of segment dy there (without the cell across the x edge) and its
        // wrapped cell.
        const bool seam = wm == 1;
        const int r = __builtin_amdgcn_readfirstlane(cy);
        const uint32_t Mx = (uint32_t)g.Mx;
        const uint32_t cxA = (uint32_t)__builtin_amdgcn_readfirstlane(cx);
        const uint32_t cxB = (uint32_t)__builtin_amdgcn_readlane(cx, 63);
        // first row of segment dy = k - 1 and the y shift of its images
        uint32_t srow[3];
        float soy[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int y = r + k - 1;
            srow[k] = (uint32_t)(y < 0 ? y + g.My : (y >= g.My ? y - g.My : y));
            soy[k] = y < 0 ? -g.Lyf : (y >= g.My ? g.Lyf : 0.0f);
        }
        // bounds of the nine segments, lanes 0..17: [lo, hi) of segments
        // dy = -1, 0, 1, then of the cells 0 of the lanes in column Mx-1
        // (rows r-1 .. r+1), then of the cells Mx-1 of the lanes in column 0
        // (rows r .. r+2 for a seam wave, r-1 .. r+1 for a one-row wave);
        // empty when the wave has no such lane
        const bool has_r = seam || cxB == Mx - 1u, has_l = seam || cxA == 0u;
        uint32_t bi = 0;
        if (lane < 6) {
            const uint32_t rb = sel3(lane >> 1, srow[0], srow[1], srow[2]) * Mx;
            bi = (lane & 1) ? rb + (seam ? Mx + cxB + 2u : min(cxB + 2u, Mx))
                            : rb + (cxA >= 1u ? cxA - 1u : 0u);
        } else if (lane < 12) {
            const uint32_t rb = sel3((lane - 6) >> 1, srow[0], srow[1], srow[2]) * Mx;
            bi = has_r ? rb + (uint32_t)(lane & 1) : 0u;
        } else if (lane < 18) {
            const int j = (lane - 12) >> 1;
            const uint32_t row = seam ? (uint32_t)(r + j) : sel3(j, srow[0], srow[1], srow[2]);
            bi = has_l ? row * Mx + Mx - 1u + (uint32_t)(lane & 1) : 0u;
        }
        const uint32_t bv = lane < 18 ? a.start[bi] : 0u;
        constexpr uint32_t kGap = kUnroll - 1;
        uint32_t slo[9], slen[9], spos[9];
        uint32_t T = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            slo[k] = __builtin_amdgcn_readlane(bv, 2 * k);
            slen[k] = __builtin_amdgcn_readlane(bv, 2 * k + 1) - slo[k];
            spos[k] = T;
            T += slen[k] + (slen[k] != 0u ? kGap : 0u);   // an empty segment is never read
        }
        // each lane's window bounds: the starts of cells cx-1 .. cx+2 of its
        // three rows (one 16-byte load per row, 4-byte aligned; for a lane in
        // column 0 or Mx-1 the first or last start lies in the row before or
        // after, never outside the array: see wrap_tile)
        uint4 sr[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int y = cy + k - 1;
            const uint32_t row = (uint32_t)(y < 0 ? y + g.My : (y >= g.My ? y - g.My : y));
            __builtin_memcpy(&sr[k], a.start + row * Mx + (uint32_t)cx - 1u, 16);
        }
        o0 = sr[1].y;
        o1 = sr[1].z;
        const bool right = cx == g.Mx - 1, left = cx == 0;   // lanes at an x edge
        constexpr int kTileIters = (kCap + 63) / 64;
        constexpr int kIdIters = (kTileIdCap + 63) / 64;
        // A lane's walk of segment k -- staged in LDS from position mpos on
        // (records from slo_k) -- and of its wrapped cell: the records from
        // wj on, wlen of them, staged from position wpos on when cells is
        // set, else read from the cell-sorted array.
        auto walk = [&](const uint4& s, uint32_t slo_k, uint32_t mpos, float oy, uint32_t wj,
                        uint32_t wlen, uint32_t wpos, bool cells) {
            const uint32_t mlo = left ? s.y : s.x;
            const uint32_t mhi = right ? s.z : s.w;
            const Cand* w = L.tile + (mpos + (mlo - slo_k));
            for (uint32_t q = 0; q < mhi - mlo; q += kUnroll) {
                Cand Qv[kUnroll];
                uint32_t jv[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    Qv[u] = w[q + u];
                    jv[u] = mlo + q + (uint32_t)u;
                }
                int32_t bc = 0, bs = 0;
                uint32_t bn = 0;
                if (oy == 0.0f)
                    add_batch<false, kNvm>(Qv, kUnroll, xs, ys, a, me, jv, bc, bs, bn);
                else
                    add_batch_shift<kNvm>(Qv, mhi - mlo - q, xs, ys, 0.0f, oy, a, me, jv, bc, bs, bn);
                Cf += bc;
                Sf += bs;
                n += bn;
            }
            const float ox = right ? g.Lxf : -g.Lxf;
            const Cand* ww = L.tile + wpos;
            for (uint32_t q = 0; q < wlen; q += kUnroll) {
                Cand Qv[kUnroll];
                uint32_t jv[kUnroll];
                if (cells) {
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        Qv[u] = ww[q + u];
                        jv[u] = wj + q + (uint32_t)u;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        jv[u] = wj + min(q + (uint32_t)u, wlen - 1u);
                        Qv[u] = a.candB[jv[u]];
                    }
                }
                int32_t bc = 0, bs = 0;
                uint32_t bn = 0;
                add_batch_shift<kNvm>(Qv, wlen - q, xs, ys, ox, oy, a, me, jv, bc, bs, bn);
                Cf += bc;
                Sf += bs;
                n += bn;
            }
        };
        const uint32_t T3 = spos[3];   // the end of the three range segments
        if (T3 <= (uint32_t)kCap && slen[1] <= (uint32_t)kTileIdCap) {
            // the three range segments: every load in flight, then the stores
            // (dense waves: the six one-cell segments stay in the cell-sorted
            // array when the nine do not fit together)
            const bool cells = T <= (uint32_t)kCap;
            Cand v[kTileIters];
            uint32_t idv[kIdIters];
#pragma unroll
            for (int k = 0; k < kTileIters; ++k) {
                const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                const bool in0 = e < slen[0];
                const bool in1 = e >= spos[1] && e < spos[1] + slen[1];
                const bool in2 = e >= spos[2] && e < spos[2] + slen[2];
                const uint32_t j = in0 ? slo[0] + e
                                       : in1 ? slo[1] + (e - spos[1]) : slo[2] + (e - spos[2]);
                v[k] = make_int4(0x7FC00000, 0x7FC00000, 0, 0);
                if (in0 || in1 || in2) v[k] = a.candB[j];
            }
#pragma unroll
            for (int k = 0; k < kIdIters; ++k) {
                const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                idv[k] = e < slen[1] ? a.oriB[slo[1] + e].y : 0u;
            }
#pragma unroll
            for (int k = 0; k < kTileIters; ++k) {
                const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                if (e < T3) L.tile[e] = v[k];
            }
#pragma unroll
            for (int k = 0; k < kIdIters; ++k) {
                const uint32_t e = (uint32_t)lane + 64u * (uint32_t)k;
                if (e < slen[1]) L.ids[e] = idv[k];
            }
            // the six one-cell segments (a few records each)
            for (uint32_t e = T3 + (uint32_t)lane; cells && e < T; e += 64u) {
                // the segment of position e: the last one starting at or before it
                uint32_t lo = slo[3], len = slen[3], pos = spos[3];
#pragma unroll
                for (int q = 4; q < 9; ++q) {
                    const bool in = e >= spos[q];
                    lo = in ? slo[q] : lo;
                    len = in ? slen[q] : len;
                    pos = in ? spos[q] : pos;
                }
                const uint32_t i = e - pos;
                Cand w = make_int4(0x7FC00000, 0x7FC00000, 0, 0);
                if (i < len) w = a.candB[lo + i];
                L.tile[e] = w;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            __builtin_amdgcn_s_setprio(0);
            // rank by id in the own cell, from the staged ids of segment 0
            const uint32_t r0 = o0 - slo[1], r1 = o1 - slo[1];
            for (uint32_t e = r0; e < r1; e += 4) {
                uint32_t iv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) iv[u] = L.ids[min(e + (uint32_t)u, r1 - 1u)];
#pragma unroll
                for (int u = 0; u < 4; ++u) rank += (e + (uint32_t)u < r1 && iv[u] < idi) ? 1u : 0u;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint32_t wlen = right ? slen[3 + k] : (left ? slen[6 + k] : 0u);
                walk(sr[k], slo[k], spos[k], soy[k], right ? slo[3 + k] : slo[6 + k], wlen,
                     right ? spos[3 + k] : spos[6 + k], cells);
            }
        } else {
            // the range segments do not fit the tile: the same walk from the
            // cell-sorted array
            rank = rank_staged(a, L, o0, o1, idi, lane);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint32_t mlo = left ? sr[k].y : sr[k].x;
                const uint32_t mhi = right ? sr[k].z : sr[k].w;
                for (uint32_t q = 0; q < mhi - mlo; q += kUnroll) {
                    Cand Qv[kUnroll];
                    uint32_t jv[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        jv[u] = mlo + min(q + (uint32_t)u, mhi - mlo - 1u);
                        Qv[u] = a.candB[jv[u]];
                    }
                    int32_t bc = 0, bs = 0;
                    uint32_t bn = 0;
                    add_batch_shift<kNvm>(Qv, mhi - mlo - q, xs, ys, 0.0f, soy[k], a, me, jv, bc,
                                          bs, bn);
                    Cf += bc;
                    Sf += bs;
                    n += bn;
                }
                const uint32_t wlen = right ? slen[3 + k] : (left ? slen[6 + k] : 0u);
                const uint32_t wj = right ? slo[3 + k] : slo[6 + k];
                const float ox = right ? g.Lxf : -g.Lxf;
                for (uint32_t q = 0; q < wlen; q += kUnroll) {
                    Cand Qv[kUnroll];
                    uint32_t jv[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        jv[u] = wj + min(q + (uint32_t)u, wlen - 1u);
                        Qv[u] = a.candB[jv[u]];
                    }
                    int32_t bc = 0, bs = 0;
                    uint32_t bn = 0;
                    add_batch_shift<kNvm>(Qv, wlen - q, xs, ys, ox, soy[k], a, me, jv, bc, bs, bn);
                    Cf += bc;
                    Sf += bs;
                    n += bn;
                }
            }
        }
        n -= 1;   // the particle itself
    } else {
        // A wave holding an edge particle: every lane walks its three rows,
        // each row as two runs of cells, run A and run B, seen through an
        // image map x -> s x + o (s = +-1).  Away from the x edges run A is
        // the three cells and run B is empty; in the first column run A is
        // the cell beyond the edge (wrapped or mirrored) and run B cells 0, 1;
        // in the last column run A is the two cells and run B the one beyond.
        o0 = a.start[own];
        o1 = a.start[own + 1];
        rank = rank_staged(a, L, o0, o1, idi, lane);
        const double xd = (double)xs, yd = (double)ys;
        int ga0 = cx - 1, ga1 = cx + 2, gb0 = 0, gb1 = 0;
        float sa = 1.0f, oa = 0.0f, sb = 1.0f, ob = 0.0f;
        if (cx == 0) {
            ga0 = BX ? 0 : g.Mx - 1;
            ga1 = ga0 + 1;
            image_map(BX ? kImgMirror0 : kImgMinusL, g.Lxf, sa, oa);
            gb0 = 0;
            gb1 = 2;
        } else if (cx == g.Mx - 1) {
            ga0 = cx - 1;
            ga1 = cx + 1;
            gb0 = BX ? g.Mx - 1 : 0;
            gb1 = gb0 + 1;
            image_map(BX ? kImgMirrorL : kImgPlusL, g.Lxf, sb, ob);
        }
        // the bounds of all three rows' runs first: their loads in flight at once
        uint32_t ejA[3], elA[3], ejB[3], elB[3];
        float esy[3], eoy[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int gy, yc;
            map_axis(cy + k - 1, g.My, BY, gy, yc);
            image_map(yc, g.Lyf, esy[k], eoy[k]);
            const uint32_t row = (uint32_t)gy * (uint32_t)g.Mx;
            ejA[k] = a.start[row + ga0];
            elA[k] = a.start[row + ga1];
            ejB[k] = a.start[row + gb0];
            elB[k] = a.start[row + gb1];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float sy = esy[k], oy = eoy[k];
            const uint32_t jA = ejA[k], lA = elA[k] - jA;
            const uint32_t jB = ejB[k], lB = elB[k] - jB;
            const uint32_t tot = lA + lB;
            for (uint32_t q = 0; q < tot; q += kEdgeUnroll) {
                Cand Qv[kEdgeUnroll];
                uint32_t jv[kEdgeUnroll];
#pragma unroll
                for (int u = 0; u < kEdgeUnroll; ++u) {
                    const uint32_t qq = min(q + (uint32_t)u, tot - 1u);
                    jv[u] = qq < lA ? jA + qq : jB + (qq - lA);
                    Qv[u] = a.candB[jv[u]];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < kEdgeUnroll; ++u) {
                    const bool inA = q + (uint32_t)u < lA;
                    const float s_x = inA ? sa : sb, o_x = inA ? oa : ob;
                    const float xj = __int_as_float(Qv[u].x), yj = __int_as_float(Qv[u].y);
                    const float dx = (s_x * xj + o_x) - xs;
                    const float dy = (sy * yj + oy) - ys;
                    const float d2 = dx * dx + dy * dy;
                    // an image of the particle itself is no neighbour (j != i)
                    const bool self_image =
                        jv[u] == p && (s_x < 0.0f || o_x != 0.0f || sy < 0.0f || oy != 0.0f);
                    bool hit = q + (uint32_t)u < tot && !self_image && d2 <= a.r2_hi_edge;
                    if (hit && !(d2 < a.r2_lo_edge))
                        hit = exact_hit_map(xj, yj, s_x, o_x, sy, oy, xd, yd, g.R2);
                    if (hit) {
                        ++n;
                        // mirrors: theta -> pi - theta (x), theta -> -theta (y);
                        // for the o-th harmonic the x mirror is (-1)^o e^{-i o theta}
                        const bool mx = s_x < 0.0f, my = sy < 0.0f;
                        const bool even = RULE == 1 && (a.m.order & 1) == 0;
                        int32_t cz = (mx && !even) ? -Qv[u].z : Qv[u].z;
                        int32_t cw = (my != (mx && even)) ? -Qv[u].w : Qv[u].w;
                        if (kNvm) nvm_orient(cz, cw, me, mx, my, true, jv[u], a);
                        Cf += cz;
                        Sf += cw;
                    }
                }
            }
        }
        n -= 1;   // the particle itself
    }
    __builtin_amdgcn_s_setprio(0);
    if (live)
        finish_particle<RULE, BX, BY>(a, xs, ys, __uint_as_float(O.x), P.z, P.w, idi, n, Cf, Sf,
                                      o0 + rank, step, meas, acc);
}

// One workgroup of THREADS lanes of the neighbour kernel: particles
// b * THREADS + tid of the system a (cell-sorted positions), then the
// measured sums of its waves (slot group by the wave's first particle / 64,
// whatever THREADS is).
template <int RULE, int BX, int BY, int THREADS = kNbrThreads>
__device__ __forceinline__ void nbr_block(const NbrArgs& a, uint32_t b, uint32_t step, bool meas,
                                          WaveLds<tile_cap(RULE)>* lds) {
    const uint32_t p = b * THREADS + threadIdx.x;
    Acc acc{0, 0, 0, 0, 0};
    const bool live = p < a.N;
    nbr_particle<RULE, BX, BY>(a, live ? p : a.N - 1u, live, step, meas, lds[threadIdx.x >> 6],
                               acc);
    if (!meas) return;
    // per-wave measured sums into the fixed-point slots (integer atomics);
    // a lane's terms are one unit vector (|c|, |s| <= 2^27) and its n
    // (n can exceed 2^27 only in huge dense systems: then it is summed apart)
    const bool big_n = __any(acc.sn > (1ll << 27));
    const long long sn_big = big_n ? wave_sum_i64(acc.sn) : 0;
    int32_t v[5] = {(int32_t)acc.sc, (int32_t)acc.ss, big_n ? 0 : (int32_t)acc.sn,
                    (int32_t)acc.sc2, (int32_t)acc.ss2};
    const int lane = threadIdx.x & 63;
    const long long tot = wave_sums5(v, lane);
    if (lane < 40 && (lane & 7) == 0) {
        const int q = lane >> 3;
        const uint32_t wg = b * (THREADS / 64) + (threadIdx.x >> 6);
        atomicAdd(reinterpret_cast<unsigned long long*>(
                      &a.obs_slots[(wg % kObsSlots) * kObsWords + q]),
                  (unsigned long long)(tot + (q == 2 ? sn_big : 0)));
    }
}

// Seven waves per SIMD for the VM and Langevin rules: the register budget
// (at most 72 VGPRs and 94 SGPRs) the compiler is held to; the wrapped-tile
// path would otherwise take more SGPRs, and at the hardware's allocation
// (trap registers included) only six waves would fit.
template <int RULE, int BX, int BY>
__global__ __launch_bounds__(kNbrThreads) __attribute__((amdgpu_waves_per_eu(RULE == 2 ? 5 : 7)))
void k_nbr(NbrArgs a) {
    __shared__ WaveLds<tile_cap(RULE)> lds[kNbrThreads / 64];
    const uint32_t step = a.step_dev ? *a.step_dev : a.step;
    // the block index is uniform: kept in a scalar register
    const uint32_t blk = __builtin_amdgcn_readfirstlane(
        xcd_spread(a.N) ? xcd_block_spread() : xcd_block());
    nbr_block<RULE, BX, BY>(a, blk, step, a.obs_slots != nullptr, lds);
}

// Batched form: one launch for every replica of a batch.  Workgroup gb
// belongs to replica blk2rep[gb] and is that replica's block
// gb - blk0[replica]; each replica's arguments come from the table.  The
// workgroups stay dealt round-robin over the XCDs (no renumbering): the
// replicas differ in density, hence in work per block, and contiguous runs
// would load the XCDs unevenly.  The step is read from the device (the batched sort advances
// it), so a captured sequence of steps replays with the right noise.
template <int RULE, int BX, int BY, int THREADS>
__global__ __launch_bounds__(THREADS) void k_nbr_b(const NbrArgs* __restrict__ tab,
                                                   const uint32_t* __restrict__ blk2rep,
                                                   const uint32_t* __restrict__ blk0,
                                                   const uint32_t* __restrict__ d_step,
                                                   int32_t meas) {
    __shared__ WaveLds<tile_cap(RULE)> lds[THREADS / 64];
    const uint32_t gb = blockIdx.x;
    const uint32_t r = blk2rep[gb];
    nbr_block<RULE, BX, BY, THREADS>(tab[r], gb - blk0[r], *d_step, meas != 0, lds);
}

// ---------------------------------------------------------------------------
// Histograms of the measured state (Sec. 3.4): the neighbour kernel wrote
// each particle's (angle bin | n bin << 16); each workgroup counts its share
// in LDS and adds its counts to the 64-bit accumulators.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kHistThreads) void k_hist(const uint32_t* __restrict__ bins, uint32_t N,
                                                       uint32_t bt, uint32_t bn,
                                                       unsigned long long* acc_t,
                                                       unsigned long long* acc_n) {
    __shared__ uint32_t ht[kHistMaxBins], hn[kHistMaxBins];
    for (uint32_t k = threadIdx.x; k < bt; k += kHistThreads) ht[k] = 0u;
    for (uint32_t k = threadIdx.x; k < bn; k += kHistThreads) hn[k] = 0u;
    __syncthreads();
    const uint32_t i0 = blockIdx.x * (uint32_t)(kHistThreads * kHistItems);
    for (int u = 0; u < kHistItems; ++u) {
        const uint32_t i = i0 + (uint32_t)u * kHistThreads + threadIdx.x;
        if (i < N) {
            const uint32_t w = bins[i];
            atomicAdd(&ht[w & 0xFFFFu], 1u);
            atomicAdd(&hn[w >> 16], 1u);
        }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < bt; k += kHistThreads)
        if (ht[k]) atomicAdd(&acc_t[k], (unsigned long long)ht[k]);
    for (uint32_t k = threadIdx.x; k < bn; k += kHistThreads)
        if (hn[k]) atomicAdd(&acc_n[k], (unsigned long long)hn[k]);
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers.  With a (start, stop) event pair the events ride on the
// kernel's own dispatch (hipExtLaunchKernelGGL), so they time the kernel
// itself and add no packets to the stream.
// ---------------------------------------------------------------------------
namespace {
template <typename K, typename... Args>
hipError_t launch(K kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                  Args... args) {
    if (e0 && e1)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t value, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

hipError_t launch_init(Cand* cand, Ori* ori, uint32_t N, const Geom& g, uint32_t key0,
                       uint32_t key1, uint32_t replica, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3((N + 255) / 256), dim3(256), 0, st, cand, ori, N, g, key0,
                       key1, replica);
    return hipGetLastError();
}

hipError_t launch_prepare(Cand* cand, const Ori* ori, uint2* kslot, uint32_t* key,
                          uint32_t* count, uint32_t N, const Geom& g, int order, hipStream_t st) {
    hipLaunchKernelGGL(k_prepare, dim3((N + 255) / 256), dim3(256), 0, st, cand, ori, kslot, key,
                       count, N, g, order);
    return hipGetLastError();
}

hipError_t launch_sort(const Cand* candA, const Ori* oriA, const uint32_t* key,
                       const uint32_t* start_old, uint32_t* start_new, Cand* candB, Ori* oriB,
                       uint32_t ncells, uint32_t N, uint32_t Mx, uint32_t My, uint32_t w,
                       int periodic_y, const uint32_t* tile_count, uint32_t* tile_clear,
                       const uint32_t* tile_offset, long long* obs_slots, double* obs_acc,
                       double* series, int fold, int slot, uint32_t* err, uint32_t* step_dev,
                       hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    SortArgs a;
    a.step_dev = step_dev;
    a.candA = candA;
    a.oriA = oriA;
    a.key = key;
    a.start_old = start_old;
    a.start_new = start_new;
    a.candB = candB;
    a.oriB = oriB;
    a.tile_count = tile_count;
    a.tile_clear = tile_clear;
    a.tile_offset = tile_offset;
    a.obs_slots = obs_slots;
    a.obs_acc = obs_acc;
    a.series = series;
    a.err = err;
    a.nblocks = sort_blocks(ncells);
    a.ncells = ncells;
    a.N = N;
    a.Mx = Mx;
    a.My = My;
    a.w = w;
    a.periodic_y = periodic_y ? 1u : 0u;
    a.fold = fold;
    a.slot = slot;
    return launch(k_sort, dim3(a.nblocks), dim3(kSortThreads), st, e0, e1, a);
}

hipError_t launch_tile_offsets(const uint32_t* tile_count, uint32_t nblocks, uint32_t* offset,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_tile_offsets, dim3(1), dim3(1024), 0, st, tile_count, nblocks, offset);
    return hipGetLastError();
}

SortArgs sort_args(const Cand* candA, const Ori* oriA, const uint32_t* key,
                   const uint32_t* start_old, uint32_t* start_new, Cand* candB, Ori* oriB,
                   uint32_t ncells, uint32_t N, uint32_t Mx, uint32_t My, uint32_t w,
                   int periodic_y, const uint32_t* tile_count, uint32_t* tile_clear,
                   long long* obs_slots, double* obs_acc, double* series, int slot,
                   uint32_t* err) {
    SortArgs a;
    a.step_dev = nullptr;
    a.candA = candA;
    a.oriA = oriA;
    a.key = key;
    a.start_old = start_old;
    a.start_new = start_new;
    a.candB = candB;
    a.oriB = oriB;
    a.tile_count = tile_count;
    a.tile_clear = tile_clear;
    a.tile_offset = nullptr;
    a.obs_slots = obs_slots;
    a.obs_acc = obs_acc;
    a.series = series;
    a.err = err;
    a.nblocks = sort_blocks(ncells);
    a.ncells = ncells;
    a.N = N;
    a.Mx = Mx;
    a.My = My;
    a.w = w;
    a.periodic_y = periodic_y ? 1u : 0u;
    a.fold = 0;
    a.slot = slot;
    return a;
}

hipError_t launch_sort_batch(const SortArgs* tab, const uint32_t* blk2rep, const uint32_t* blk0,
                             uint32_t nblocks, uint32_t* d_step, int fold, hipStream_t st,
                             hipEvent_t e0, hipEvent_t e1) {
    return launch(k_sort_b, dim3(nblocks), dim3(kSortThreads), st, e0, e1, tab, blk2rep, blk0,
                  d_step, (int32_t)fold);
}

template <int THREADS>
hipError_t launch_nbr_batch_t(const NbrArgs* tab, const uint32_t* blk2rep, const uint32_t* blk0,
                              uint32_t nblocks, const uint32_t* d_step, int32_t m, int sel,
                              hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid(nblocks), block(THREADS);
#define AAP_NBR_B(R_, X_, Y_) \
    launch(k_nbr_b<R_, X_, Y_, THREADS>, grid, block, st, e0, e1, tab, blk2rep, blk0, d_step, m)
    switch (sel) {
    case 0: return AAP_NBR_B(0, 0, 0);
    case 1: return AAP_NBR_B(0, 0, 1);
    case 2: return AAP_NBR_B(0, 1, 0);
    case 3: return AAP_NBR_B(0, 1, 1);
    case 4: return AAP_NBR_B(1, 0, 0);
    case 5: return AAP_NBR_B(1, 0, 1);
    case 6: return AAP_NBR_B(1, 1, 0);
    case 7: return AAP_NBR_B(1, 1, 1);
    case 8: return AAP_NBR_B(2, 0, 0);
    case 9: return AAP_NBR_B(2, 0, 1);
    case 10: return AAP_NBR_B(2, 1, 0);
    default: return AAP_NBR_B(2, 1, 1);
    }
#undef AAP_NBR_B
}

hipError_t launch_nbr_batch(const NbrArgs* tab, const uint32_t* blk2rep, const uint32_t* blk0,
                            uint32_t nblocks, const uint32_t* d_step, int meas, int rule,
                            int bx, int by, int threads, hipStream_t st, hipEvent_t e0,
                            hipEvent_t e1) {
    if (rule < 0 || rule > 2) return hipErrorInvalidValue;
    const int sel = rule * 4 + (bx ? 2 : 0) + (by ? 1 : 0);
    const int32_t m = meas ? 1 : 0;
    switch (threads) {
    case 64: return launch_nbr_batch_t<64>(tab, blk2rep, blk0, nblocks, d_step, m, sel, st, e0, e1);
    case 128:
        return launch_nbr_batch_t<128>(tab, blk2rep, blk0, nblocks, d_step, m, sel, st, e0, e1);
    case 256:
        return launch_nbr_batch_t<256>(tab, blk2rep, blk0, nblocks, d_step, m, sel, st, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scan(uint32_t* count, uint32_t* start, uint32_t ncells,
                       unsigned long long* status, unsigned long long* ticket,
                       long long* obs_slots, double* obs_acc, double* series, int fold,
                       int slot, uint32_t N, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const uint32_t nb = scan_blocks(ncells);
    return launch(k_scan, dim3(nb), dim3(kScanThreads), st, e0, e1, count, start, ncells, status,
                  ticket, nb, obs_slots, obs_acc, series, (int32_t)fold, (int32_t)slot, N);
}

hipError_t launch_scatter(const Cand* candA, const Ori* oriA, const uint2* kslot,
                          const uint32_t* start, Cand* candB, Ori* oriB, uint32_t N,
                          uint32_t* err, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const uint32_t per = 256u * kScatterItems;
    return launch(k_scatter, dim3((N + per - 1) / per), dim3(256), st, e0, e1, candA, oriA, kslot,
                  start, candB, oriB, N, err);
}

hipError_t launch_nbr(const NbrArgs& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid((a.N + kNbrThreads - 1) / kNbrThreads), block(kNbrThreads);
    if (a.m.rule < 0 || a.m.rule > 2) return hipErrorInvalidValue;
    const int sel = a.m.rule * 4 + (a.g.bx ? 2 : 0) + (a.g.by ? 1 : 0);
    switch (sel) {
    case 0: return launch(k_nbr<0, 0, 0>, grid, block, st, e0, e1, a);
    case 1: return launch(k_nbr<0, 0, 1>, grid, block, st, e0, e1, a);
    case 2: return launch(k_nbr<0, 1, 0>, grid, block, st, e0, e1, a);
    case 3: return launch(k_nbr<0, 1, 1>, grid, block, st, e0, e1, a);
    case 4: return launch(k_nbr<1, 0, 0>, grid, block, st, e0, e1, a);
    case 5: return launch(k_nbr<1, 0, 1>, grid, block, st, e0, e1, a);
    case 6: return launch(k_nbr<1, 1, 0>, grid, block, st, e0, e1, a);
    case 7: return launch(k_nbr<1, 1, 1>, grid, block, st, e0, e1, a);
    case 8: return launch(k_nbr<2, 0, 0>, grid, block, st, e0, e1, a);
    case 9: return launch(k_nbr<2, 0, 1>, grid, block, st, e0, e1, a);
    case 10: return launch(k_nbr<2, 1, 0>, grid, block, st, e0, e1, a);
    default: return launch(k_nbr<2, 1, 1>, grid, block, st, e0, e1, a);
    }
}

hipError_t launch_hist(const uint32_t* bins, uint32_t N, uint32_t bt, uint32_t bn,
                       unsigned long long* acc_t, unsigned long long* acc_n, hipStream_t st) {
    const uint32_t per = (uint32_t)(kHistThreads * kHistItems);
    hipLaunchKernelGGL(k_hist, dim3((N + per - 1) / per), dim3(kHistThreads), 0, st, bins, N, bt,
                       bn, acc_t, acc_n);
    return hipGetLastError();
}

hipError_t launch_obs(long long* obs_slots, double* obs_acc, double* series, int slot,
                      uint32_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_obs, dim3(1), dim3(64), 0, st, obs_slots, obs_acc, series,
                       (int32_t)slot, N);
    return hipGetLastError();
}

}  // namespace aap

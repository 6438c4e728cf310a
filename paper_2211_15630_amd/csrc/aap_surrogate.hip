// Learned field surrogate on gfx950: the coarse-grained fields of a particle
// state and a small periodic convolutional network that advances them,
// trained and run with bf16 matrix-core products (v_mfma_f32_16x16x16_bf16,
// fp32 accumulation).
//
// Fields (the measured quantities of Sec. 3.4, resolved in space): on a
// G x G grid of square bins of side L / G, the number density rho and the
// polarisation density p = sum e^{i theta} per unit area; a particle's bin
// is floor(x G / L) in binary64 from its binary32 coordinate, clamped to
// G - 1.  The unit vectors are the stored 2^-27 fixed-point ones, summed
// exactly in integers.
//
// Network: input u = (rho / rho0 - 1, p_x / rho0, p_y / rho0) zero-padded to
// 16 channels, three 3x3 convolutions with ReLU (16 -> 32 -> 32 -> 32) and a
// linear one (32 -> 16, three channels used); prediction = u + output.
// Periodic (circular) padding, channel-last activations [b][y][x][c] in
// bf16 between layers, weights in bf16, fp32 master weights and Adam.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "aap.h"
#include "aap_internal.h"

using namespace aap;

namespace {

int sfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

#define AAP_SHIP(call)                                                         \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return sfail(AAP_EHIP, "%s: %s", #call, hipGetErrorString(e_));    \
    } while (0)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kCin0 = 16, kHid = 32, kCout3 = 16;   // padded input, hidden, padded output
constexpr int kLayers = 4;
constexpr int kLayerCin[kLayers] = {kCin0, kHid, kHid, kHid};
constexpr int kLayerCout[kLayers] = {kHid, kHid, kHid, kCout3};
constexpr double kFixInvS = 1.0 / 134217728.0;   // 2^-27

// bfloat16 bits of a binary32 value, rounded to nearest, ties to even
__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bool bf16_positive(uint16_t h) {
    return h != 0 && (h & 0x8000u) == 0;
}

// ---------------------------------------------------------------------------
// fields of a state
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// One particle per lane.  A stepped state is stored in cell order, so the 64
// particles of a wave fall into two or three bins: the wave sums the lanes
// of one bin at a time (exact int64 sums) and one lane adds them to the
// bin's accumulators, instead of 64 atomics to one address per instruction.
// Any order is correct; a shuffled state only takes more rounds.
__global__ void k_fields_acc(const Cand* __restrict__ cand, uint32_t N, double scale, int G,
                             unsigned* __restrict__ cnt, unsigned long long* __restrict__ sc,
                             unsigned long long* __restrict__ ss) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int k = -1;
    long long cz = 0, cw = 0;
    if (i < N) {
        const Cand c = cand[i];
        const double ux = (double)__int_as_float(c.x) * scale;
        const double uy = (double)__int_as_float(c.y) * scale;
        int bx = ux > 0.0 ? (int)ux : 0;
        int by = uy > 0.0 ? (int)uy : 0;
        bx = bx < G - 1 ? bx : G - 1;
        by = by < G - 1 ? by : G - 1;
        k = by * G + bx;
        cz = c.z;
        cw = c.w;
    }
    bool todo = k >= 0;
    for (;;) {
        const unsigned long long pend = __ballot(todo);
        if (pend == 0) break;
        const int leader = __ffsll((long long)pend) - 1;
        const int key = __builtin_amdgcn_readlane(k, leader);
        const bool mine = todo && k == key;
        const unsigned long long m = __ballot(mine);
        const long long sz = wave_sum_i64(mine ? cz : 0);
        const long long sw = wave_sum_i64(mine ? cw : 0);
        if (lane == leader) {
            atomicAdd(&cnt[key], (unsigned)__popcll(m));
            atomicAdd(&sc[key], (unsigned long long)sz);
            atomicAdd(&ss[key], (unsigned long long)sw);
        }
        todo = todo && !mine;
    }
}

__global__ void k_fields_fin(const unsigned* __restrict__ cnt,
                             const unsigned long long* __restrict__ sc,
                             const unsigned long long* __restrict__ ss, int G, double inv_area,
                             float* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= G * G) return;
    out[k] = (float)((double)cnt[k] * inv_area);
    out[G * G + k] = (float)((double)(long long)sc[k] * kFixInvS * inv_area);
    out[2 * G * G + k] = (float)((double)(long long)ss[k] * kFixInvS * inv_area);
}

__global__ void k_zero32(uint32_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------------------
// network input and output
// ---------------------------------------------------------------------------
// fields [nb][3][G][G] -> u fp32 [nb][G][G][3], x0 bf16 [nb][G][G][16]
__global__ void k_prep(const float* __restrict__ f, int nb, int G, float inv_rho0,
                       float* __restrict__ u, uint16_t* __restrict__ x0) {
    const size_t P = (size_t)nb * G * G;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const size_t GG = (size_t)G * G;
    const size_t b = p / GG, q = p % GG;
    const float u0 = f[(b * 3 + 0) * GG + q] * inv_rho0 - 1.0f;
    const float u1 = f[(b * 3 + 1) * GG + q] * inv_rho0;
    const float u2 = f[(b * 3 + 2) * GG + q] * inv_rho0;
    u[p * 3 + 0] = u0;
    u[p * 3 + 1] = u1;
    u[p * 3 + 2] = u2;
    uint16_t* o = x0 + p * kCin0;
    o[0] = bf16_rne(u0);
    o[1] = bf16_rne(u1);
    o[2] = bf16_rne(u2);
#pragma unroll
    for (int c = 3; c < kCin0; ++c) o[c] = 0;
}

// prediction fp32 [nb][G][G][3] -> fields [nb][3][G][G]
__global__ void k_unprep(const float* __restrict__ pred, int nb, int G, float rho0,
                         float* __restrict__ f) {
    const size_t P = (size_t)nb * G * G;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const size_t GG = (size_t)G * G;
    const size_t b = p / GG, q = p % GG;
    f[(b * 3 + 0) * GG + q] = rho0 * (pred[p * 3 + 0] + 1.0f);
    f[(b * 3 + 1) * GG + q] = rho0 * pred[p * 3 + 1];
    f[(b * 3 + 2) * GG + q] = rho0 * pred[p * 3 + 2];
}

// ---------------------------------------------------------------------------
// 3x3 periodic convolution on the matrix cores
//
// One wave computes `tiles` runs of 16 pixels of one row for all COUT
// output channels: an implicit product with K = 9 taps x CIN channels, in
// steps of 16 channels of one tap.  The wave holds every weight operand in
// registers (9 x CIN/16 x COUT/16 fragments) for all its pixel runs.  Operand layout of v_mfma_f32_16x16x16_bf16:
// lane l holds A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16],
// j = 0..3, and returns D[4 (l / 16) + j][l % 16].  Here A rows are pixels,
// B columns output channels, K input channels: each lane loads 4
// consecutive channels (8 bytes) of one pixel and of one weight row.
//
// MODE 0: + bias, ReLU, bf16 out [.., COUT]
// MODE 1: + bias, fp32 prediction resid + out for channels 0..2
// MODE 2: gradient of the layer input (weights given flipped and
//         transposed): times the ReLU mask of that input, bf16 out
// ---------------------------------------------------------------------------
struct ConvArgs {
    const uint16_t* in;      // [nb][G][G][CIN]
    const uint16_t* w;       // [9][COUT][CIN]
    const float* bias;       // [COUT] (modes 0, 1)
    const uint16_t* mask;    // [nb][G][G][COUT] (mode 2)
    const float* resid;      // [nb][G][G][3] (mode 1)
    uint16_t* out16;         // modes 0, 2
    float* out32;            // mode 1: [nb][G][G][3]
    int nb, G;
    int tiles;               // 16-pixel runs per wave (set by the launcher)
};

// Up to kConvTiles runs per wave share the wave's weight registers; small
// batches take fewer so that the launch still has kConvWaves waves.
constexpr int kConvTiles = 4;
constexpr size_t kConvWaves = 2048;

// Epilogue of a 16-pixel run starting at pixel index p0 (of [nb][G][G]):
// lane (mrow, kq) holds output channels n 16 + mrow of pixels p0 + kq + j.
template <int COUT, int MODE>
__device__ __forceinline__ void conv_store(const ConvArgs& a, const f32x4 (&acc)[COUT / 16],
                                           size_t p0, int mrow, int kq) {
#pragma unroll
    for (int n = 0; n < COUT / 16; ++n) {
        const int co = n * 16 + mrow;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t o = p0 + kq + j;
            float v = acc[n][j];
            if (MODE == 0) {
                v += a.bias[co];
                v = v > 0.f ? v : 0.f;
                a.out16[o * COUT + co] = bf16_rne(v);
            } else if (MODE == 1) {
                v += a.bias[co];
                if (co < 3) a.out32[o * 3 + co] = a.resid[o * 3 + co] + v;
            } else {
                if (!bf16_positive(a.mask[o * COUT + co])) v = 0.f;
                a.out16[o * COUT + co] = bf16_rne(v);
            }
        }
    }
}

// The same epilogue for COUT = 32 and modes 0 and 2 through a wave-private
// LDS tile [16 pixels][32 channels]: the values are written there in the
// product's layout, then each lane moves 8 channels of one pixel (16 bytes)
// at once, so that the stores (and the mask loads of mode 2) are whole,
// consecutive 16-byte pieces.
template <int MODE>
__device__ __forceinline__ void conv_store_tile(const ConvArgs& a, const f32x4 (&acc)[2], size_t p0,
                                                int mrow, int kq, int lane, uint16_t* tile) {
    constexpr int COUT = 32;
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int co = n * 16 + mrow;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float v = acc[n][j];
            if (MODE == 0) {
                v += a.bias[co];
                v = v > 0.f ? v : 0.f;
            }
            tile[(kq + j) * COUT + co] = bf16_rne(v);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int q = lane >> 2, g = lane & 3;   // pixel, group of 8 channels
    uint4 v = *reinterpret_cast<const uint4*>(tile + q * COUT + g * 8);
    const size_t o = (p0 + q) * COUT + g * 8;
    if (MODE == 2) {
        const uint4 m = *reinterpret_cast<const uint4*>(a.mask + o);
        const uint32_t mw[4] = {m.x, m.y, m.z, m.w};
        uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t keep_lo = bf16_positive((uint16_t)(mw[k] & 0xFFFFu)) ? 0x0000FFFFu : 0u;
            const uint32_t keep_hi = bf16_positive((uint16_t)(mw[k] >> 16)) ? 0xFFFF0000u : 0u;
            vw[k] &= keep_lo | keep_hi;
        }
        v = make_uint4(vw[0], vw[1], vw[2], vw[3]);
    }
    *reinterpret_cast<uint4*>(a.out16 + o) = v;
    // the tile is rewritten by the next run of this wave only after every
    // lane has read it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
    constexpr int CB = CIN / 16, NT = COUT / 16;
    const int lane = threadIdx.x & 63;
    const int G = a.G;
    const int xtiles = G / 16;
    const int groups = (xtiles + a.tiles - 1) / a.tiles;
    const size_t wave = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= (size_t)a.nb * G * groups) return;
    const int grp = (int)(wave % groups);
    const int y = (int)((wave / groups) % G);
    const int b = (int)(wave / ((size_t)groups * G));
    const int mrow = lane & 15, kq = 4 * (lane >> 4);
    bf16x4 Bf[9][CB][NT];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int n = 0; n < NT; ++n)
                Bf[t][cb][n] = *reinterpret_cast<const bf16x4*>(
                    a.w + ((size_t)(t * COUT + n * 16 + mrow)) * CIN + cb * 16 + kq);
    const int xt1 = min(xtiles, (grp + 1) * a.tiles);
    for (int xt = grp * a.tiles; xt < xt1; ++xt) {
        const int x0 = xt * 16;
        f32x4 acc[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            const int yy = (y + dy + G) % G;
            const int xx = (x0 + mrow + dx + G) % G;
            const uint16_t* row = a.in + ((size_t)(b * G + yy) * G + xx) * CIN + kq;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const bf16x4 A = *reinterpret_cast<const bf16x4*>(row + cb * 16);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bf[t][cb][n], acc[n], 0,
                                                                       0, 0);
            }
        }
        conv_store<COUT, MODE>(a, acc, (size_t)(b * G + y) * G + x0, mrow, kq);
    }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[t][ci][co] = sum over pixels p of
// x[p + offset(t)][ci] dy[p][co], tap t = (a, c) at offset (a - 1, c - 1),
// as matrix-core products with rows = input channels, columns = output
// channels, K = pixels.  Substituting q = p + c - 1, the sum is over q of
// x[row y + a - 1][q][ci] dy[row y][q - c + 1][co].
//
// Workgroup `chunk` covers the output rows [r0, r1) of the batch (row
// r = b G + y) in segments of up to kWgSeg pixels.  For each row it holds in
// LDS, transposed (pixel fastest), the input rows y - 1, y, y + 1 (a ring of
// three, reused by consecutive rows) and three copies of the dy row shifted
// by c - 1, so that both operands of every product are 4 consecutive pixels
// of one channel: one 8-byte LDS read per lane.  Wave w owns the (mb, nt)
// tile pair w % PAIRS for all nine taps and the K steps of parity
// w / PAIRS; with two waves per pair their sums are added in a fixed order.
// Each workgroup writes its partial sums; a second kernel adds the chunks in
// order.
// ---------------------------------------------------------------------------
constexpr int kWgSeg = 128;       // pixels of a row segment
constexpr int kWgChunks = 512;    // workgroups (partial sums) at most

// Transposes 4 pixels x 8 channels (channel-last, 16 bytes per pixel) into
// dst[ch * kWgSeg + 0..3] (pixel fastest, 8-byte stores).
__device__ __forceinline__ void stage4x8(const uint16_t* const (&src)[4], uint16_t* dst) {
    uint4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = *reinterpret_cast<const uint4*>(src[k]);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        uint32_t h[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t w = (j >> 1) == 0 ? v[k].x : (j >> 1) == 1 ? v[k].y
                             : (j >> 1) == 2 ? v[k].z : v[k].w;
            h[k] = (j & 1) ? (w >> 16) : (w & 0xFFFFu);
        }
        *reinterpret_cast<uint2*>(dst + j * kWgSeg) =
            make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ x,
                                               const uint16_t* __restrict__ dy,
                                               float* __restrict__ part, int nb, int G,
                                               int nchunks) {
    constexpr int MT = CIN / 16, NT = COUT / 16, PAIRS = MT * NT, KG = 4 / PAIRS;
    static_assert(PAIRS * KG == 4, "four waves per workgroup");
    constexpr int XS = 3 * CIN * kWgSeg, DS = 3 * COUT * kWgSeg;        // bf16 elements
    constexpr int RED = (KG == 2) ? 2 * 9 * 64 * 4 * 2 : 0;            // floats as bf16 slots
    constexpr int LDS = (XS + DS) > RED ? (XS + DS) : RED;
    __shared__ __align__(16) uint16_t lds[LDS];
    uint16_t* xs = lds;             // [3][CIN][kWgSeg]
    uint16_t* ds = lds + XS;        // [3][COUT][kWgSeg]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pair = wave % PAIRS, kg = wave / PAIRS;
    const int mb = pair / NT, nt = pair % NT;
    const int chunk = blockIdx.x;
    const long rows = (long)nb * G;
    const long r0 = rows * chunk / nchunks, r1 = rows * (chunk + 1) / nchunks;
    const int row16 = lane & 15, kq = 4 * (lane >> 4);
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int x0 = 0; x0 < G; x0 += kWgSeg) {
        const int Ls = min(kWgSeg, G - x0);      // a multiple of 16
        long tag[3] = {-1, -1, -1};              // input row held by each ring slot
        for (long r = r0; r < r1; ++r) {
            const int b = (int)(r / G), y = (int)(r % G);
            long need[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) need[a] = (long)b * G + (y + a - 1 + G) % G;
            // ring slots: keep the rows still needed, stage the others
            int slot[3];
            bool fresh[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                slot[a] = -1;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (slot[a] < 0 && tag[k] == need[a]) slot[a] = k;
                fresh[a] = slot[a] < 0;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (!fresh[a]) continue;
                for (int k = 0; k < 3; ++k) {
                    const bool used = (slot[0] == k) || (slot[1] == k) || (slot[2] == k);
                    if (!used) {
                        slot[a] = k;
                        break;
                    }
                }
            }
            __syncthreads();   // the previous row's products are done with the LDS
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (!fresh[a]) continue;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (slot[a] == k) tag[k] = need[a];
                const uint16_t* src = x + (size_t)need[a] * G * CIN;
                const int items = (Ls / 4) * (CIN / 8);
                for (int i = tid; i < items; i += 256) {
                    const int g = i % (CIN / 8), q0 = 4 * (i / (CIN / 8));
                    const uint16_t* px[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) px[k] = src + (size_t)(x0 + q0 + k) * CIN + 8 * g;
                    stage4x8(px, xs + (slot[a] * CIN + 8 * g) * kWgSeg + q0);
                }
            }
            {
                const uint16_t* src = dy + (size_t)r * G * COUT;
                const int per = (Ls / 4) * (COUT / 8);
                for (int i = tid; i < 3 * per; i += 256) {
                    const int c = i / per, e = i % per;
                    const int g = e % (COUT / 8), q0 = 4 * (e / (COUT / 8));
                    const uint16_t* px[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        px[k] = src + (size_t)((x0 + q0 + k - c + 1 + G) % G) * COUT + 8 * g;
                    stage4x8(px, ds + (c * COUT + 8 * g) * kWgSeg + q0);
                }
            }
            __syncthreads();
            for (int ks = kg; ks < Ls / 16; ks += KG) {
                const int k0 = ks * 16 + kq;
                bf16x4 A[3], Bv[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    A[a] = *reinterpret_cast<const bf16x4*>(
                        xs + (slot[a] * CIN + mb * 16 + row16) * kWgSeg + k0);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    Bv[c] = *reinterpret_cast<const bf16x4*>(
                        ds + (c * COUT + nt * 16 + row16) * kWgSeg + k0);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        acc[a * 3 + c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                            A[a], Bv[c], acc[a * 3 + c], 0, 0, 0);
            }
        }
    }
    float* o = part + (size_t)chunk * 9 * CIN * COUT;
    if (KG == 2) {
        f32x4* red = reinterpret_cast<f32x4*>(lds);     // [PAIRS][9][64]
        __syncthreads();
        if (kg == 1) {
#pragma unroll
            for (int t = 0; t < 9; ++t) red[(pair * 9 + t) * 64 + lane] = acc[t];
        }
        __syncthreads();
        if (kg == 1) return;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[t] += red[(pair * 9 + t) * 64 + lane];
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            o[((size_t)t * CIN + mb * 16 + kq + j) * COUT + nt * 16 + row16] = acc[t][j];
}

// grad[i] = sum over chunks of part[chunk][i], i < n, in a fixed order:
// 32 outputs per workgroup; thread group cg (0..7) sums the chunks
// c = cg, cg + 8, ... in turn, then group 0 adds the eight group sums in
// order.
constexpr int kSumGroups = 8;
__global__ __launch_bounds__(256) void k_chunk_sum(const float* __restrict__ part, int nchunks,
                                                   size_t n, float* __restrict__ grad) {
    __shared__ float red[kSumGroups][32];
    const int il = threadIdx.x & 31, cg = threadIdx.x >> 5;
    const size_t i = (size_t)blockIdx.x * 32 + il;
    float s = 0.f;
    if (i < n) {
#pragma unroll 8
        for (int c = cg; c < nchunks; c += kSumGroups) s += part[(size_t)c * n + i];
    }
    red[cg][il] = s;
    __syncthreads();
    if (cg == 0 && i < n) {
        float t = red[0][il];
#pragma unroll
        for (int k = 1; k < kSumGroups; ++k) t += red[k][il];
        grad[i] = t;
    }
}

// bias gradient, partial sums: part[chunk][co] = sum over the chunk's
// pixels of dy[p][co].  Thread tid reads 8 consecutive channels (16 bytes)
// of every (256 / (COUT / 8))-th pixel, then a fixed tree over the pixel
// offsets.  COUT is 16 or 32; dy is 16-byte aligned.
__global__ __launch_bounds__(256) void k_bgrad(const uint16_t* __restrict__ dy, size_t P,
                                               int COUT, int nchunks, float* __restrict__ part) {
    __shared__ float s[8][256];
    const int tid = threadIdx.x;
    const int groups = COUT / 8;
    const int g = tid % groups, pofs = tid / groups, stride = 256 / groups;
    const size_t p0 = P * blockIdx.x / nchunks, p1 = P * (blockIdx.x + 1) / nchunks;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (size_t p = p0 + pofs; p < p1; p += stride) {
        const uint4 v = *reinterpret_cast<const uint4*>(dy + p * COUT + g * 8);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc[2 * k] += __uint_as_float(w[k] << 16);            // channel 2k: low half
            acc[2 * k + 1] += __uint_as_float(w[k] & 0xFFFF0000u);  // channel 2k + 1
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j][tid] = acc[j];
    __syncthreads();
    for (int d = stride / 2; d > 0; d >>= 1) {
        if (pofs < d) {
#pragma unroll
            for (int j = 0; j < 8; ++j) s[j][tid] += s[j][tid + d * groups];
        }
        __syncthreads();
    }
    if (pofs == 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) part[(size_t)blockIdx.x * COUT + g * 8 + j] = s[j][tid];
    }
}

// loss: per pixel the squared error of the three channels against the
// target fields; dout = 2 (pred - target) / n in bf16 (channels 3..15 zero);
// per-block partial sums in binary64 (fixed tree)
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ pred,
                                              const float* __restrict__ tf, int nb, int G,
                                              float inv_rho0, float scale,
                                              uint16_t* __restrict__ dout,
                                              double* __restrict__ part) {
    __shared__ double s[256];
    const size_t P = (size_t)nb * G * G;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (p < P) {
        const size_t GG = (size_t)G * G;
        const size_t b = p / GG, q = p % GG;
        const float t0 = tf[(b * 3 + 0) * GG + q] * inv_rho0 - 1.0f;
        const float t1 = tf[(b * 3 + 1) * GG + q] * inv_rho0;
        const float t2 = tf[(b * 3 + 2) * GG + q] * inv_rho0;
        const float d0 = pred[p * 3 + 0] - t0;
        const float d1 = pred[p * 3 + 1] - t1;
        const float d2 = pred[p * 3 + 2] - t2;
        e = (double)d0 * d0 + (double)d1 * d1 + (double)d2 * d2;
        uint16_t* o = dout + p * kCout3;
        o[0] = bf16_rne(scale * d0);
        o[1] = bf16_rne(scale * d1);
        o[2] = bf16_rne(scale * d2);
#pragma unroll
        for (int c = 3; c < kCout3; ++c) o[c] = 0;
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Adam (Kingma and Ba, 2015) on the fp32 master parameters; c1 = lr /
// (1 - b1^t), c2 = 1 / (1 - b2^t)
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float b1, float b2, float c1, float c2,
                       float eps) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= c1 * mi / (sqrtf(vi * c2) + eps);
}

// bf16 weights of one layer from the master [t][ci][co]: forward layout
// wf[t][co][ci], gradient-of-input layout wb[t][ci][co] = w[8 - t][ci][co]
__global__ void k_pack(const float* __restrict__ w, int CIN, int COUT, uint16_t* __restrict__ wf,
                       uint16_t* __restrict__ wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * CIN * COUT) return;
    const int t = i / (CIN * COUT), r = i % (CIN * COUT), ci = r / COUT, co = r % COUT;
    const uint16_t h = bf16_rne(w[i]);
    wf[((size_t)t * COUT + co) * CIN + ci] = h;
    if (wb) wb[((size_t)(8 - t) * CIN + ci) * COUT + co] = h;
}

template <typename K, typename... Args>
hipError_t go(K kernel, size_t threads, int block, hipStream_t st, Args... args) {
    if (threads == 0) return hipSuccess;
    const size_t blocks = (threads + block - 1) / block;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(block), 0, st, args...);
    return hipGetLastError();
}

}  // namespace

namespace aap {

size_t fields_scratch_bytes(int G) {
    return (size_t)G * G * (4 + 8 + 8);
}

hipError_t launch_fields(const Cand* cand, uint32_t N, double L, int G, void* scratch,
                         float* out, hipStream_t st) {
    unsigned* cnt = (unsigned*)scratch;
    unsigned long long* sc = (unsigned long long*)((char*)scratch + (size_t)G * G * 4);
    unsigned long long* ss = sc + (size_t)G * G;
    const size_t words = fields_scratch_bytes(G) / 4;
    hipError_t e = go(k_zero32, words < 1024 * 256 ? words : 1024 * 256, 256, st,
                      (uint32_t*)scratch, words);
    if (e != hipSuccess) return e;
    e = go(k_fields_acc, N, 256, st, cand, N, (double)G / L, G, cnt, sc, ss);
    if (e != hipSuccess) return e;
    const double side = L / G;
    return go(k_fields_fin, (size_t)G * G, 256, st, (const unsigned*)cnt,
              (const unsigned long long*)sc, (const unsigned long long*)ss, G,
              1.0 / (side * side), out);
}

}  // namespace aap

// ---------------------------------------------------------------------------
// the network object
// ---------------------------------------------------------------------------
struct aap_cnn {
    int G = 0, maxb = 0;
    hipStream_t st = nullptr;
    size_t nparam = 0;
    size_t off_w[kLayers], off_b[kLayers];
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t* wf[kLayers] = {};
    uint16_t* wb[kLayers] = {};
    float* u = nullptr;             // [maxb][G][G][3]
    uint16_t* x0 = nullptr;         // [maxb][G][G][16]
    uint16_t* act[3] = {};          // [maxb][G][G][32]
    float* pred = nullptr;          // [maxb][G][G][3]
    uint16_t* dout = nullptr;       // [maxb][G][G][16]
    uint16_t* dact[2] = {};         // [maxb][G][G][32]
    float* part = nullptr;          // [chunks][9][32][32] gradient partials
    double* lpart = nullptr;        // loss partials
    int adam_t = 0;
};

namespace {

constexpr int kBiasChunks = 512;   // bias-gradient partials (fit in the weight partials' buffer)
static_assert(kBiasChunks * kHid <= kWgChunks * 9 * kHid * kHid, "bias partials exceed the buffer");

struct CnnLayout {
    size_t p, m, v, grad, wf[kLayers], wb[kLayers], u, x0, act[3], pred, dout, dact[2], part,
        lpart, bytes;
};

size_t cnn_nparam(size_t* off_w = nullptr, size_t* off_b = nullptr) {
    size_t n = 0;
    for (int k = 0; k < kLayers; ++k) {
        if (off_w) off_w[k] = n;
        n += (size_t)9 * kLayerCin[k] * kLayerCout[k];
        if (off_b) off_b[k] = n;
        n += (size_t)kLayerCout[k];
    }
    return n;
}

int cnn_layout(int G, int maxb, CnnLayout* L) {
    if (G < 16 || G > 1024 || (G % 16) != 0)
        return sfail(AAP_EINVAL, "grid side must be a multiple of 16 in [16, 1024] (got %d)", G);
    if (maxb < 1 || maxb > 1024) return sfail(AAP_EINVAL, "batch must be in [1, 1024] (got %d)", maxb);
    const size_t P = (size_t)maxb * G * G;
    const size_t np = cnn_nparam();
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = (o + bytes + 255) & ~(size_t)255; return at; };
    L->p = take(np * 4);
    L->m = take(np * 4);
    L->v = take(np * 4);
    L->grad = take(np * 4);
    for (int k = 0; k < kLayers; ++k) {
        L->wf[k] = take((size_t)9 * kLayerCin[k] * kLayerCout[k] * 2);
        L->wb[k] = take((size_t)9 * kLayerCin[k] * kLayerCout[k] * 2);
    }
    L->u = take(P * 3 * 4);
    L->x0 = take(P * kCin0 * 2);
    for (int k = 0; k < 3; ++k) L->act[k] = take(P * kHid * 2);
    L->pred = take(P * 3 * 4);
    L->dout = take(P * kCout3 * 2);
    for (int k = 0; k < 2; ++k) L->dact[k] = take(P * kHid * 2);
    L->part = take((size_t)kWgChunks * 9 * kHid * kHid * 4);
    L->lpart = take(((P + 255) / 256) * 8);
    L->bytes = o;
    return AAP_OK;
}

int cnn_pack(aap_cnn* c) {
    for (int k = 0; k < kLayers; ++k)
        AAP_SHIP(go(k_pack, (size_t)9 * kLayerCin[k] * kLayerCout[k], 256, c->st,
                    (const float*)(c->p + c->off_w[k]), kLayerCin[k], kLayerCout[k], c->wf[k],
                    k > 0 ? c->wb[k] : (uint16_t*)nullptr));
    return AAP_OK;
}

// LDS form for large launches.  A workgroup computes kConvRows output rows
// of a segment of up to kConvSeg pixels: it stages the kConvRows + 2 input
// rows of the segment plus one halo pixel on each side (periodic) in LDS,
// channel-last with kConvPad extra channels per pixel so that the 16 pixels
// of a fragment spread over the banks, and each wave computes pairs of
// 16-pixel runs of those rows with its weights in registers.
constexpr int kConvRows = 4;
constexpr int kConvSeg = 128;
constexpr int kConvPad = 8;

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv_lds(ConvArgs a) {
    constexpr int CB = CIN / 16, NT = COUT / 16, CP = CIN + kConvPad;
    constexpr int PIX = kConvSeg + 2;
    __shared__ __align__(16) uint16_t xs[(kConvRows + 2) * PIX * CP];
    constexpr bool kTileOut = COUT == 32 && MODE != 1;
    __shared__ __align__(16) uint16_t outt[kTileOut ? 4 * 16 * 32 : 8];   // per wave [16][32]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = a.G;
    const int nseg = (G + kConvSeg - 1) / kConvSeg;
    const int rgroups = G / kConvRows;
    const int seg = (int)(blockIdx.x % nseg);
    const int rg = (int)((blockIdx.x / nseg) % rgroups);
    const int b = (int)(blockIdx.x / ((size_t)nseg * rgroups));
    const int x0 = seg * kConvSeg, Ls = min(kConvSeg, G - x0);   // Ls: a multiple of 16
    const int y0 = rg * kConvRows;
    // stage rows y0 - 1 .. y0 + kConvRows, pixels x0 - 1 .. x0 + Ls (16 bytes a thread)
    {
        constexpr int C8 = CIN / 8;
        const int items = (kConvRows + 2) * (Ls + 2) * C8;
        for (int i = tid; i < items; i += 256) {
            const int g = i % C8, pr = i / C8;
            const int px = pr % (Ls + 2), r = pr / (Ls + 2);
            const int yy = (y0 + r - 1 + G) % G, xx = (x0 + px - 1 + G) % G;
            const uint4 v = *reinterpret_cast<const uint4*>(
                a.in + ((size_t)(b * G + yy) * G + xx) * CIN + g * 8);
            *reinterpret_cast<uint4*>(xs + (r * PIX + px) * CP + g * 8) = v;
        }
    }
    const int mrow = lane & 15, kq = 4 * (lane >> 4);
    bf16x4 Bf[9][CB][NT];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int n = 0; n < NT; ++n)
                Bf[t][cb][n] = *reinterpret_cast<const bf16x4*>(
                    a.w + ((size_t)(t * COUT + n * 16 + mrow)) * CIN + cb * 16 + kq);
    __syncthreads();
    // two runs of a row at a time (run pairs: Ls / 16 is even unless Ls = 16,
    // then the second run of the pair is skipped), so that each wave keeps
    // 2 NT independent accumulation chains in flight
    const int rr = Ls / 16, pairs = kConvRows * ((rr + 1) / 2);
    for (int item = wave; item < pairs; item += 4) {
        const int r = item / ((rr + 1) / 2), xr = (item % ((rr + 1) / 2)) * 32;
        const bool two = xr + 16 < Ls;
        f32x4 acc[2][NT];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[h][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            const uint16_t* row = xs + ((r + 1 + dy) * PIX + xr + mrow + dx + 1) * CP + kq;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const bf16x4 A0 = *reinterpret_cast<const bf16x4*>(row + cb * 16);
                const bf16x4 A1 = *reinterpret_cast<const bf16x4*>(row + 16 * CP + cb * 16);
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    acc[0][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A0, Bf[t][cb][n],
                                                                          acc[0][n], 0, 0, 0);
                    acc[1][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A1, Bf[t][cb][n],
                                                                          acc[1][n], 0, 0, 0);
                }
            }
        }
        const size_t p0 = (size_t)(b * G + y0 + r) * G + x0 + xr;
        if constexpr (kTileOut) {
            uint16_t* tile = outt + wave * 16 * 32;
            conv_store_tile<MODE>(a, acc[0], p0, mrow, kq, lane, tile);
            if (two) conv_store_tile<MODE>(a, acc[1], p0 + 16, mrow, kq, lane, tile);
        } else {
            conv_store<COUT, MODE>(a, acc[0], p0, mrow, kq);
            if (two) conv_store<COUT, MODE>(a, acc[1], p0 + 16, mrow, kq);
        }
    }
}

template <int CIN, int COUT, int MODE>
hipError_t conv(ConvArgs a, hipStream_t st) {
    // large launches: the LDS form, when it still has kConvWaves waves
    const size_t lds_wgs = (size_t)a.nb * (a.G / kConvRows) *
                           ((a.G + kConvSeg - 1) / kConvSeg);
    if (lds_wgs * 4 >= kConvWaves)
        return go(k_conv_lds<CIN, COUT, MODE>, lds_wgs * 256, 256, st, a);
    const size_t runs = (size_t)a.nb * a.G * (a.G / 16);
    const size_t t = runs / kConvWaves;
    a.tiles = t < 1 ? 1 : t > (size_t)kConvTiles ? kConvTiles : (int)t;
    const size_t groups = (size_t)(a.G / 16 + a.tiles - 1) / a.tiles;
    const size_t waves = (size_t)a.nb * a.G * groups;
    return go(k_conv<CIN, COUT, MODE>, waves * 64, 256, st, a);
}

int cnn_forward(aap_cnn* c, const float* fields, int nb, double rho0) {
    const int G = c->G;
    const size_t P = (size_t)nb * G * G;
    AAP_SHIP(go(k_prep, P, 256, c->st, fields, nb, G, (float)(1.0 / rho0), c->u, c->x0));
    ConvArgs a{};
    a.nb = nb;
    a.G = G;
    a.in = c->x0;
    a.w = c->wf[0];
    a.bias = c->p + c->off_b[0];
    a.out16 = c->act[0];
    AAP_SHIP((conv<kCin0, kHid, 0>(a, c->st)));
    for (int k = 1; k < 3; ++k) {
        a.in = c->act[k - 1];
        a.w = c->wf[k];
        a.bias = c->p + c->off_b[k];
        a.out16 = c->act[k];
        AAP_SHIP((conv<kHid, kHid, 0>(a, c->st)));
    }
    a.in = c->act[2];
    a.w = c->wf[3];
    a.bias = c->p + c->off_b[3];
    a.out16 = nullptr;
    a.resid = c->u;
    a.out32 = c->pred;
    AAP_SHIP((conv<kHid, kCout3, 1>(a, c->st)));
    return AAP_OK;
}

template <int CIN, int COUT>
int wgrad(aap_cnn* c, const uint16_t* x, const uint16_t* dy, int nb, int layer) {
    const long rows = (long)nb * c->G;
    const int nchunks = (int)(rows < kWgChunks ? rows : kWgChunks);
    hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(nchunks), dim3(256), 0, c->st, x, dy, c->part,
                       nb, c->G, nchunks);
    AAP_SHIP(hipGetLastError());
    const size_t n = (size_t)9 * CIN * COUT;
    hipLaunchKernelGGL(k_chunk_sum, dim3((unsigned)((n + 31) / 32)), dim3(256), 0, c->st,
                       (const float*)c->part, nchunks, n, c->grad + c->off_w[layer]);
    AAP_SHIP(hipGetLastError());
    hipLaunchKernelGGL(k_bgrad, dim3(kBiasChunks), dim3(256), 0, c->st, dy,
                       (size_t)nb * c->G * c->G, COUT, kBiasChunks, c->part);
    AAP_SHIP(hipGetLastError());
    hipLaunchKernelGGL(k_chunk_sum, dim3((unsigned)((COUT + 31) / 32)), dim3(256), 0, c->st,
                       (const float*)c->part, kBiasChunks, (size_t)COUT,
                       c->grad + c->off_b[layer]);
    AAP_SHIP(hipGetLastError());
    return AAP_OK;
}

}  // namespace

extern "C" {

size_t aap_cnn_param_count(void) { return cnn_nparam(); }

int aap_fields_scratch_bytes(int32_t G, size_t* bytes) {
    if (!bytes) return sfail(AAP_EINVAL, "bytes is NULL");
    if (G < 1 || G > 4096) return sfail(AAP_EINVAL, "grid side must be in [1, 4096]");
    *bytes = fields_scratch_bytes(G);
    return AAP_OK;
}

int aap_cnn_workspace_bytes(int32_t G, int32_t max_batch, size_t* bytes) {
    if (!bytes) return sfail(AAP_EINVAL, "bytes is NULL");
    CnnLayout L;
    const int rc = cnn_layout(G, max_batch, &L);
    if (rc) return rc;
    *bytes = L.bytes;
    return AAP_OK;
}

int aap_cnn_create(int32_t G, int32_t max_batch, void* d_workspace, size_t bytes,
                   void* hip_stream, aap_cnn** out) {
    if (!out) return sfail(AAP_EINVAL, "out is NULL");
    *out = nullptr;
    CnnLayout L;
    int rc = cnn_layout(G, max_batch, &L);
    if (rc) return rc;
    if (!d_workspace) return sfail(AAP_EINVAL, "workspace is NULL");
    if (((uintptr_t)d_workspace & 255) != 0)
        return sfail(AAP_ENOMEM, "workspace not 256-B aligned");
    if (bytes < L.bytes)
        return sfail(AAP_ENOMEM, "workspace of %zu B is smaller than the %zu B needed", bytes,
                     L.bytes);
    aap_cnn* c = new (std::nothrow) aap_cnn;
    if (!c) return sfail(AAP_ENOMEM, "host allocation failed");
    char* ws = (char*)d_workspace;
    c->G = G;
    c->maxb = max_batch;
    c->st = (hipStream_t)hip_stream;
    c->nparam = cnn_nparam(c->off_w, c->off_b);
    c->p = (float*)(ws + L.p);
    c->m = (float*)(ws + L.m);
    c->v = (float*)(ws + L.v);
    c->grad = (float*)(ws + L.grad);
    for (int k = 0; k < kLayers; ++k) {
        c->wf[k] = (uint16_t*)(ws + L.wf[k]);
        c->wb[k] = (uint16_t*)(ws + L.wb[k]);
    }
    c->u = (float*)(ws + L.u);
    c->x0 = (uint16_t*)(ws + L.x0);
    for (int k = 0; k < 3; ++k) c->act[k] = (uint16_t*)(ws + L.act[k]);
    c->pred = (float*)(ws + L.pred);
    c->dout = (uint16_t*)(ws + L.dout);
    for (int k = 0; k < 2; ++k) c->dact[k] = (uint16_t*)(ws + L.dact[k]);
    c->part = (float*)(ws + L.part);
    c->lpart = (double*)(ws + L.lpart);
    // parameters, moments and gradients start at zero
    rc = [&]() -> int {
        AAP_SHIP(go(k_zero32, 1024 * 256, 256, c->st, (uint32_t*)(ws + L.p),
                    (L.wf[0] - L.p) / 4));
        return cnn_pack(c);
    }();
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return AAP_OK;
}

int aap_cnn_destroy(aap_cnn* c) {
    if (!c) return sfail(AAP_EINVAL, "handle is NULL");
    (void)hipStreamSynchronize(c->st);
    delete c;
    return AAP_OK;
}

int aap_cnn_set_params(aap_cnn* c, const float* host, size_t count) {
    if (!c || !host) return sfail(AAP_EINVAL, "NULL argument");
    if (count != c->nparam)
        return sfail(AAP_EINVAL, "expected %zu parameters (got %zu)", c->nparam, count);
    AAP_SHIP(hipMemcpyAsync(c->p, host, count * 4, hipMemcpyHostToDevice, c->st));
    AAP_SHIP(go(k_zero32, 1024 * 256, 256, c->st, (uint32_t*)c->m, count));
    AAP_SHIP(go(k_zero32, 1024 * 256, 256, c->st, (uint32_t*)c->v, count));
    c->adam_t = 0;
    const int rc = cnn_pack(c);
    if (rc) return rc;
    AAP_SHIP(hipStreamSynchronize(c->st));
    return AAP_OK;
}

int aap_cnn_get_params(aap_cnn* c, float* host, size_t count) {
    if (!c || !host) return sfail(AAP_EINVAL, "NULL argument");
    if (count != c->nparam)
        return sfail(AAP_EINVAL, "expected %zu parameters (got %zu)", c->nparam, count);
    AAP_SHIP(hipMemcpyAsync(host, c->p, count * 4, hipMemcpyDeviceToHost, c->st));
    AAP_SHIP(hipStreamSynchronize(c->st));
    return AAP_OK;
}

int aap_cnn_forward(aap_cnn* c, const float* d_in, int32_t nb, double rho0, float* d_out) {
    if (!c || !d_in || !d_out) return sfail(AAP_EINVAL, "NULL argument");
    if (nb < 1 || nb > c->maxb) return sfail(AAP_EINVAL, "batch %d outside [1, %d]", nb, c->maxb);
    if (!(rho0 > 0.0) || !std::isfinite(rho0)) return sfail(AAP_EINVAL, "rho0 must be > 0");
    const int rc = cnn_forward(c, d_in, nb, rho0);
    if (rc) return rc;
    AAP_SHIP(go(k_unprep, (size_t)nb * c->G * c->G, 256, c->st, (const float*)c->pred, nb, c->G,
                (float)rho0, d_out));
    return AAP_OK;
}

int aap_cnn_train_step(aap_cnn* c, const float* d_in, const float* d_target, int32_t nb,
                       double rho0, float lr, double* loss) {
    if (!c || !d_in || !d_target) return sfail(AAP_EINVAL, "NULL argument");
    if (nb < 1 || nb > c->maxb) return sfail(AAP_EINVAL, "batch %d outside [1, %d]", nb, c->maxb);
    if (!(rho0 > 0.0) || !std::isfinite(rho0)) return sfail(AAP_EINVAL, "rho0 must be > 0");
    if (!(lr >= 0.f) || !std::isfinite(lr)) return sfail(AAP_EINVAL, "learning rate must be >= 0");
    int rc = cnn_forward(c, d_in, nb, rho0);
    if (rc) return rc;
    const int G = c->G;
    const size_t P = (size_t)nb * G * G;
    const size_t nblk = (P + 255) / 256;
    const double n = (double)P * 3.0;
    AAP_SHIP(go(k_loss, P, 256, c->st, (const float*)c->pred, d_target, nb, G,
                (float)(1.0 / rho0), (float)(2.0 / n), c->dout, c->lpart));
    // layer 3 (32 -> 16, linear)
    rc = wgrad<kHid, kCout3>(c, c->act[2], c->dout, nb, 3);
    if (rc) return rc;
    ConvArgs a{};
    a.nb = nb;
    a.G = G;
    a.in = c->dout;
    a.w = c->wb[3];
    a.mask = c->act[2];
    a.out16 = c->dact[0];
    AAP_SHIP((conv<kCout3, kHid, 2>(a, c->st)));
    // layers 2, 1 (32 -> 32, ReLU)
    int cur = 0;
    for (int k = 2; k >= 1; --k) {
        rc = wgrad<kHid, kHid>(c, c->act[k - 1], c->dact[cur], nb, k);
        if (rc) return rc;
        a.in = c->dact[cur];
        a.w = c->wb[k];
        a.mask = c->act[k - 1];
        a.out16 = c->dact[1 - cur];
        AAP_SHIP((conv<kHid, kHid, 2>(a, c->st)));
        cur = 1 - cur;
    }
    // layer 0 (16 -> 32)
    rc = wgrad<kCin0, kHid>(c, c->x0, c->dact[cur], nb, 0);
    if (rc) return rc;
    // Adam
    c->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const double c1 = (double)lr / (1.0 - std::pow(b1, c->adam_t));
    const double c2 = 1.0 / (1.0 - std::pow(b2, c->adam_t));
    AAP_SHIP(go(k_adam, c->nparam, 256, c->st, c->p, (const float*)c->grad, c->m, c->v, c->nparam,
                (float)b1, (float)b2, (float)c1, (float)c2, 1e-8f));
    rc = cnn_pack(c);
    if (rc) return rc;
    if (loss) {
        std::vector<double> part(nblk);
        AAP_SHIP(hipMemcpyAsync(part.data(), c->lpart, nblk * 8, hipMemcpyDeviceToHost, c->st));
        AAP_SHIP(hipStreamSynchronize(c->st));
        double s = 0.0;
        for (double v : part) s += v;
        *loss = s / n;
    }
    return AAP_OK;
}

int aap_cnn_debug_read(aap_cnn* c, int32_t which, void* host, size_t bytes) {
    if (!c || !host) return sfail(AAP_EINVAL, "NULL argument");
    const size_t P = (size_t)c->maxb * c->G * c->G;
    const void* src = nullptr;
    size_t have = 0;
    switch (which) {
    case 0: src = c->x0; have = P * kCin0 * 2; break;
    case 1: case 2: case 3: src = c->act[which - 1]; have = P * kHid * 2; break;
    case 4: src = c->pred; have = P * 3 * 4; break;
    case 5: src = c->grad; have = c->nparam * 4; break;
    case 6: src = c->dout; have = P * kCout3 * 2; break;
    default: return sfail(AAP_EINVAL, "unknown buffer %d", which);
    }
    if (bytes > have) return sfail(AAP_EINVAL, "buffer %d holds %zu B (asked %zu)", which, have, bytes);
    AAP_SHIP(hipMemcpyAsync(host, src, bytes, hipMemcpyDeviceToHost, c->st));
    AAP_SHIP(hipStreamSynchronize(c->st));
    return AAP_OK;
}

}  // extern "C"

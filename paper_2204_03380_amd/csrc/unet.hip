// Kernels of the learned crosstalk filter: a 3-D U-Net on channels-last
// bfloat16 activations.  Convolutions are implicit GEMMs on the gfx950
// bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16, float32 accumulation):
//
//   forward / input gradient  M = voxels, N = output channels,
//                             K = 27 taps x input channels
//   weight gradient           M = output channels, N = input channels,
//                             K = voxels (one x-segment of a row at a time)
//
// MFMA 16x16x32 operand layout (lane l, element e): A[l % 16][8 (l / 16) + e],
// B[8 (l / 16) + e][l % 16]; the 4 results of lane l are D[4 (l / 16) + e][l % 16].
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>

#include "common.h"
#include "rtm.h"
#include "unet.h"

namespace rtm {
int set_error(int code, const char *msg);
void clear_error();
}  // namespace rtm

namespace {

using rtm::kNumXcd;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float32 -> bfloat16, round to nearest even (values here are finite).
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma16(const uint4 &a, const uint4 &b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// Contiguous ranges of work items per XCD (blocks are dealt to the 8 XCDs
// round-robin): neighbouring tiles share halo rows in the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks)
{
    const int64_t per = nblocks / kNumXcd;
    return (b % kNumXcd) * per + b / kNumXcd;
}

struct ConvArgs {
    const uint16_t *x;
    const uint16_t *wt;
    const float *bias;
    const uint16_t *skip;
    float *y;
    uint16_t *r;
    uint16_t *out;
    const uint16_t *mask;  // with gout: gout = bf16(y) where mask > 0, else 0 (a ReLU gradient)
    uint16_t *gout;
    int64_t nvox;
    int d, h, w;
    int relu;
    int ych;
    int64_t nblocks;  // grid size (multiple of 8)
};

// ---------------------------------------------------------------------------
// Forward convolution (and input gradient with flipped weights).  One
// wavefront computes 64 consecutive voxels x CBW blocks of 16 output
// channels (blockIdx.y selects the blocks; CBW = COUT / 16 unless a small
// grid splits the channels over more wavefronts); the four 16-voxel row
// blocks share each weight fragment and each activation fragment feeds CBW
// MFMAs.  Every output element is the same sequence of MFMAs whatever CBW.
// ---------------------------------------------------------------------------
// The fused epilogue of a convolution for channels c0 .. c0 + 7 of voxel v
// (val: the sums before bias): bias, ReLU, the float output y, the stored
// bfloat16 value r, and out (plus the skip input), as 16-byte accesses.
template <int COUT>
__device__ __forceinline__ void epi_store8(const ConvArgs &a, int64_t v, int c0, float (&val)[8])
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        val[j] += a.bias ? a.bias[c0 + j] : 0.f;
        if (a.relu) val[j] = fmaxf(val[j], 0.f);
    }
    if (a.y) {
        if (a.ych == COUT) {
            float4 *py = reinterpret_cast<float4 *>(a.y + v * COUT + c0);
            py[0] = make_float4(val[0], val[1], val[2], val[3]);
            py[1] = make_float4(val[4], val[5], val[6], val[7]);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (c0 + j < a.ych) a.y[v * a.ych + c0 + j] = val[j];
        }
    }
    const int64_t o = v * COUT + c0;
    if (a.gout) {  // the next layer's ReLU gradient (a.ych == COUT)
        const uint4 mk = *reinterpret_cast<const uint4 *>(a.mask + o);
        const uint16_t *me = reinterpret_cast<const uint16_t *>(&mk);
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            w[q] = (uint32_t)(bf2f(me[2 * q]) > 0.f ? f2bf(val[2 * q]) : (uint16_t)0) |
                   ((uint32_t)(bf2f(me[2 * q + 1]) > 0.f ? f2bf(val[2 * q + 1]) : (uint16_t)0) << 16);
        *reinterpret_cast<uint4 *>(a.gout + o) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if (a.r) {
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = (uint32_t)f2bf(val[2 * q]) | ((uint32_t)f2bf(val[2 * q + 1]) << 16);
        *reinterpret_cast<uint4 *>(a.r + o) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if (a.out) {
        float ov[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) ov[j] = val[j];
        if (a.skip) {
            const uint4 sk = *reinterpret_cast<const uint4 *>(a.skip + o);
            const uint16_t *se = reinterpret_cast<const uint16_t *>(&sk);
#pragma unroll
            for (int j = 0; j < 8; ++j) ov[j] = val[j] + bf2f(se[j]);
        }
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = (uint32_t)f2bf(ov[2 * q]) | ((uint32_t)f2bf(ov[2 * q + 1]) << 16);
        *reinterpret_cast<uint4 *>(a.out + o) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Stages rows 2*half, 2*half + 1 of a wavefront's MFMA accumulators for one
// 16-channel block (lane (r16, g): voxels rb*16 + 4g + e of channel r16) in
// its own LDS scratch of 32 voxels x kEpiStride floats, and returns the 8
// channels 8*hh .. 8*hh + 7 of voxel vl = lane mod 32 (hh = lane / 32).
constexpr int kEpiStride = 20;  // 16 channels per voxel row, padded to spread the banks, 16-byte aligned

__device__ __forceinline__ void epi_transpose(float *scr, const f32x4 (&acc2)[2], int lane, float (&val)[8])
{
    const int r16 = lane & 15, g = lane >> 4, vl = lane & 31, hh = lane >> 5;
#pragma unroll
    for (int rbl = 0; rbl < 2; ++rbl)
#pragma unroll
        for (int e = 0; e < 4; ++e) scr[(rbl * 16 + 4 * g + e) * kEpiStride + r16] = acc2[rbl][e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float4 s0 = *reinterpret_cast<const float4 *>(scr + vl * kEpiStride + 8 * hh);
    const float4 s1 = *reinterpret_cast<const float4 *>(scr + vl * kEpiStride + 8 * hh + 4);
    val[0] = s0.x; val[1] = s0.y; val[2] = s0.z; val[3] = s0.w;
    val[4] = s1.x; val[5] = s1.y; val[6] = s1.z; val[7] = s1.w;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // reads done before the scratch is written again
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// KS > 1 splits the reduction dimension over KS wavefronts of a workgroup
// (the coarse grids, whose few wavefronts would each walk all 27*CIN/32
// chunks one after another): wavefront part p takes chunks
// [p*CPP, (p+1)*CPP), CPP = ceil(NCH/KS) (chunks past tap 26 are zero, as
// in the padded last chunk); parts 1.. hand their sums to part 0 through
// LDS, which adds them in increasing part order and runs the epilogue.
template <int CIN, int COUT, int CBW = COUT / 16, int KS = 1>
__global__ __launch_bounds__(256) void conv_fwd_kernel(ConvArgs a)
{
    static_assert(KS == 1 || KS == 2 || KS == 4, "K split of 1, 2 or 4 wavefronts");
    static_assert(KS == 1 || CBW <= 4, "the K-split hand-over holds at most four output blocks");
    constexpr int K = 27 * CIN;
    constexpr int KP = (K + 31) / 32 * 32;
    constexpr int NCH = KP / 32;
    constexpr int CB = CBW;
    const int cbase = blockIdx.y * CBW * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int part = wave % KS;
    const int r16 = lane & 15, g = lane >> 4;
    const int64_t blk = xcd_block(blockIdx.x, a.nblocks);
    const int64_t vb = (blk * (4 / KS) + wave / KS) * 64;
    const bool live = vb < a.nvox;
    if constexpr (KS == 1) {
        if (!live) return;  // whole wavefront; without a K split the kernel has no barriers
    }

    const int D = a.d, H = a.h, W = a.w;
    int vz[4], vy[4], vx[4];
    bool vin[4];
    int64_t vv[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int64_t v = vb + rb * 16 + r16;
        vin[rb] = v < a.nvox;
        vv[rb] = v;
        int64_t t = v / W;
        vx[rb] = (int)(v - t * W);
        const int64_t t2 = t / H;
        vy[rb] = (int)(t - t2 * H);
        vz[rb] = (int)(t2 % D);
    }
    f32x4 acc[4][CB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};

    const uint4 zero = {0u, 0u, 0u, 0u};
    const int64_t HW = (int64_t)H * W;
    constexpr int UF = CB <= 2 ? 4 : 2;  // narrow waves keep more activation loads in flight
    constexpr int CPP = (NCH + KS - 1) / KS;  // chunks per part
    const int kc0 = part * CPP * 32;
    if (live) {
#pragma unroll UF
        for (int j = 0; j < CPP; ++j) {
            const int kc = kc0 + 32 * j;
            const int kk = kc + 8 * g;
            const int tap = kk / CIN;
            const int ci0 = kk - tap * CIN;
            const bool tv = tap < 27;
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const int64_t off = dz * HW + (int64_t)dy * W + dx;
            uint4 A[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const bool ok = tv && vin[rb] && (unsigned)(vz[rb] + dz) < (unsigned)D &&
                                (unsigned)(vy[rb] + dy) < (unsigned)H && (unsigned)(vx[rb] + dx) < (unsigned)W;
                A[rb] = ok ? *reinterpret_cast<const uint4 *>(a.x + (vv[rb] + off) * CIN + ci0) : zero;
            }
            uint4 B[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                B[cb] = tv ? *reinterpret_cast<const uint4 *>(a.wt + (int64_t)(cbase + cb * 16 + r16) * K + kk) : zero;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(A[rb], B[cb], acc[rb][cb]);
        }
    }

    if constexpr (KS > 1) {
        // [wavefront][accumulator element][lane]: each store and load is
        // 64 consecutive floats
        __shared__ float hand[4][16 * CB][64];
        if (part > 0) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) hand[wave][(rb * CB + cb) * 4 + e][lane] = acc[rb][cb][e];
        }
        __syncthreads();
        if (part > 0 || !live) return;  // after the only barrier
#pragma unroll
        for (int p = 1; p < KS; ++p)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[rb][cb][e] += hand[wave + p][(rb * CB + cb) * 4 + e][lane];
    }

    // Epilogue through the wavefront's LDS scratch (the MFMA layout would
    // store two bytes per lane per voxel): 8 channels of one voxel per lane.
    __shared__ __attribute__((aligned(16))) float escr[4][32 * kEpiStride];
    float *scr = escr[wave];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const f32x4 acc2[2] = {acc[2 * half][cb], acc[2 * half + 1][cb]};
            float val[8];
            epi_transpose(scr, acc2, lane, val);
            const int64_t v = vb + half * 32 + (lane & 31);
            if (v < a.nvox) epi_store8<COUT>(a, v, cbase + cb * 16 + 8 * (lane >> 5), val);
        }
}

// ---------------------------------------------------------------------------
// Forward convolution with the input staged in LDS (layers of at most 32
// input and 32 output channels on grids that give enough workgroups: the
// full-resolution level).  A workgroup of four
// wavefronts owns an x-segment of 64 voxels of four consecutive y rows (one
// row per wavefront) and marches z over lz planes.  The input planes z - 1,
// z, z + 1 of the segment's halo (6 rows of 66 voxels, all channels) sit in
// a three-plane LDS ring, so every activation fragment of the 27 taps is
// read from LDS instead of L1/L2.  The next plane is fetched into registers
// while the current one is computed, then written to the ring slot that the
// previous plane left.  Each output element is the same MFMA sequence as in
// conv_fwd_kernel (same K order, same fragments), so results are equal bit
// for bit.
// ---------------------------------------------------------------------------
constexpr int kLdsX = 64, kLdsY = 4;

template <int CIN>
struct LdsTile {
    static constexpr int XW = kLdsX + 2, YW = kLdsY + 2;
    static constexpr int PLANE = YW * XW * CIN;       // bf16 elements per plane
    static constexpr int VPR = CIN / 8;               // 16-byte vectors per voxel
    static constexpr int NV = YW * XW * VPR;          // vectors per plane
    static constexpr int PER = (NV + 255) / 256;      // vectors per thread
};

// Plane z of the halo tile into registers (zeros outside the grid).
template <int CIN>
__device__ __forceinline__ void lds_fetch(const ConvArgs &a, uint4 (&v)[LdsTile<CIN>::PER], int64_t nbase, int z,
                                          int y0, int x0)
{
    using T = LdsTile<CIN>;
    const bool zin = (unsigned)z < (unsigned)a.d;
#pragma unroll
    for (int k = 0; k < T::PER; ++k) {
        const int i = threadIdx.x + 256 * k;
        const int c8 = i % T::VPR, vox = i / T::VPR;
        const int xx = vox % T::XW, yy = vox / T::XW;
        const int gx = x0 - 1 + xx, gy = y0 - 1 + yy;
        v[k] = uint4{0u, 0u, 0u, 0u};
        if (i < T::NV && zin && (unsigned)gx < (unsigned)a.w && (unsigned)gy < (unsigned)a.h)
            v[k] = *reinterpret_cast<const uint4 *>(a.x + (((nbase + z) * a.h + gy) * a.w + gx) * CIN + c8 * 8);
    }
}

template <int CIN>
__device__ __forceinline__ void lds_store(uint16_t *dst, const uint4 (&v)[LdsTile<CIN>::PER])
{
    using T = LdsTile<CIN>;
#pragma unroll
    for (int k = 0; k < T::PER; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < T::NV) *reinterpret_cast<uint4 *>(dst + (int64_t)(i / T::VPR) * CIN + (i % T::VPR) * 8) = v[k];
    }
}

// Depth of conv_fwd_lds_kernel's weight ring: the largest divisor of the
// chunk count whose fragments fit in 40 registers; 1 (no ring: each chunk
// loads its own fragments) for two output blocks over 27 chunks, where the
// unrolled march would need more registers than two waves per SIMD allow.
constexpr int lds_weight_depth(int nch, int cb)
{
    if (cb > 1 && nch > 14) return 1;
    int best = 1;
    for (int d = 1; d <= nch; ++d)
        if (nch % d == 0 && d * cb * 4 <= 40) best = d;
    return best;
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_fwd_lds_kernel(ConvArgs a, int tiles_x, int tiles_y, int tiles_z, int lz,
                                                           int64_t ntiles)
{
    using T = LdsTile<CIN>;
    constexpr int K = 27 * CIN;
    constexpr int KP = (K + 31) / 32 * 32;  // chunks past tap 26 are zero, as in conv_fwd_kernel
    constexpr int CB = COUT / 16;
    __shared__ __attribute__((aligned(16))) uint16_t ring[3 * T::PLANE];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    int64_t b = xcd_block(blockIdx.x, a.nblocks);
    if (b >= ntiles) return;  // whole workgroup, before any barrier (the grid is a multiple of 8)
    const int tx = (int)(b % tiles_x);
    b /= tiles_x;
    const int ty = (int)(b % tiles_y);
    b /= tiles_y;
    const int tz = (int)(b % tiles_z);
    const int64_t n = b / tiles_z;
    const int x0 = tx * kLdsX, y0 = ty * kLdsY, z0 = tz * lz;
    const int z1 = min(z0 + lz, a.d);
    const int64_t nbase = n * a.d;               // first plane of this sample
    const int yw = y0 + wave;                    // this wavefront's output row
    const bool row_ok = yw < a.h;
    const uint4 zero = {0u, 0u, 0u, 0u};

    // Weight fragments run PD chunks ahead of their MFMAs through a ring of
    // registers (PD divides the chunk count, so chunk c of every plane uses
    // slot c mod PD and the ring carries on from one plane to the next:
    // the weights are the same for every plane).  One load per chunk
    // waited on right away would leave each chunk waiting a full memory
    // latency.
    constexpr int NCH = KP / 32;
    constexpr int PD = lds_weight_depth(NCH, CB);
    auto load_b = [&](int c, uint4(&B)[CB]) {
        const int kk = c * 32 + 8 * g;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
            B[cb] = kk / CIN < 27 ? *reinterpret_cast<const uint4 *>(a.wt + (int64_t)(cb * 16 + r16) * K + kk) : zero;
    };
    uint4 Bq[PD][CB];
    if constexpr (PD > 1) {
#pragma unroll
        for (int i = 0; i < PD; ++i) load_b(i, Bq[i]);
    }
    uint4 next[T::PER];
    lds_fetch<CIN>(a, next, nbase, z0 - 1, y0, x0);
    lds_store<CIN>(ring + ((z0 + 2) % 3) * T::PLANE, next);
    lds_fetch<CIN>(a, next, nbase, z0, y0, x0);
    lds_store<CIN>(ring + (z0 % 3) * T::PLANE, next);
    lds_fetch<CIN>(a, next, nbase, z0 + 1, y0, x0);
    for (int z = z0; z < z1; ++z) {
        lds_store<CIN>(ring + ((z + 1) % 3) * T::PLANE, next);  // the slot plane z - 2 left
        __syncthreads();
        if (z + 1 < z1) lds_fetch<CIN>(a, next, nbase, z + 2, y0, x0);  // in flight during this plane
        f32x4 acc[4][CB];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        auto chunk = [&](int c, const uint4(&B)[CB]) {
            const int kk = c * 32 + 8 * g;
            const int tap = kk / CIN;
            const int ci0 = kk - tap * CIN;
            const bool tv = tap < 27;
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const uint16_t *pl = ring + ((z + dz + 3) % 3) * T::PLANE + ((wave + 1 + dy) * T::XW + 1 + dx) * CIN + ci0;
            uint4 A[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) A[rb] = tv ? *reinterpret_cast<const uint4 *>(pl + (rb * 16 + r16) * CIN) : zero;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(A[rb], B[cb], acc[rb][cb]);
        };
        if constexpr (PD > 1) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                chunk(c, Bq[c % PD]);
                load_b((c + PD) % NCH, Bq[c % PD]);  // chunk c + PD, of this plane or the next
                // the scheduler would otherwise sink each load to its use
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll 4
            for (int kc = 0; kc < KP; kc += 32) {
                const int kk = kc + 8 * g;
                const int tap = kk / CIN;
                const int ci0 = kk - tap * CIN;
                const bool tv = tap < 27;
                const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
                const uint16_t *pl =
                    ring + ((z + dz + 3) % 3) * T::PLANE + ((wave + 1 + dy) * T::XW + 1 + dx) * CIN + ci0;
                uint4 A[4];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    A[rb] = tv ? *reinterpret_cast<const uint4 *>(pl + (rb * 16 + r16) * CIN) : zero;
                uint4 B[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    B[cb] = tv ? *reinterpret_cast<const uint4 *>(a.wt + (int64_t)(cb * 16 + r16) * K + kk) : zero;
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(A[rb], B[cb], acc[rb][cb]);
            }
        }
        // Epilogue through LDS (the slot of plane z - 1, free once every wave
        // is past its MFMAs): 8 channels of one voxel per lane.
        __syncthreads();  // every wave is done with plane z - 1's slot
        float *scr = reinterpret_cast<float *>(ring + ((z + 2) % 3) * T::PLANE) + wave * (32 * kEpiStride);
        const int64_t vrow = ((nbase + z) * a.h + yw) * (int64_t)a.w;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const f32x4 acc2[2] = {acc[2 * half][cb], acc[2 * half + 1][cb]};
                float val[8];
                epi_transpose(scr, acc2, lane, val);
                const int xo = x0 + half * 32 + (lane & 31);
                if (row_ok && xo < a.w) epi_store8<COUT>(a, vrow + xo, cb * 16 + 8 * (lane >> 5), val);
            }
        __syncthreads();  // every wave is done with its scratch before the slot is refilled
    }
}

// ---------------------------------------------------------------------------
// Weight gradient.  Block (s, q): q = (dz, dy) neighbour-row pair, s = a
// contiguous range of output rows (n, z, y).  For each row and each
// 32-voxel x-segment the block stages dy^T [COUT][32] and three x-shifted
// copies of x^T [3][CIN][32] of the source row in LDS, then every MFMA
// reads aligned 16-byte fragments: dw[o][tap(dz,dy,dx)][i] +=
// sum_j dy[j][o] x[j + dx - 1][i].  RS row groups of WS waves: the WS waves
// of a group split the output channels, the groups split the rows.  Each
// (s, group) writes its own partial sums; a second kernel adds them in a
// fixed order.  Blocks of the centre pair also sum dy for the bias.
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
struct WgCfg {
    static constexpr int CB = COUT / 16, IB = CIN / 16;
    static constexpr int WS = CB < 4 ? CB : 4;
    static constexpr int RS = 4 / WS;
    static constexpr int CPW = CB / WS;
    static constexpr int SEG = 32;
    static constexpr int XW = SEG + 8;  // x^T row: voxels x0 - 1 .. x0 + 32, padded to whole 16-byte reads
    static constexpr int LDS_U16 = SEG * COUT + XW * CIN;  // per row group
};

struct WgArgs {
    const uint16_t *x;
    const uint16_t *dy;
    float *part;    // [S*RS][COUT][27][CIN]
    float *bpart;   // [S*RS][COUT]
    int64_t rows;   // N*D*H
    int d, h, w;
    int S;
};

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(WgArgs a)
{
    using C = WgCfg<CIN, COUT>;
    constexpr int SEG = C::SEG;
    __shared__ __attribute__((aligned(16))) uint16_t lds[C::RS * C::LDS_U16];
    const int s = blockIdx.x, q = blockIdx.y;
    const int dz = q / 3 - 1, dy = q % 3 - 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rg = wave / C::WS, wi = wave % C::WS;
    const int gt = wi * 64 + lane;  // thread index within the row group
    const int r16 = lane & 15, g = lane >> 4;
    uint16_t *dyT = lds + rg * C::LDS_U16;  // [COUT][SEG]
    uint16_t *xT = dyT + COUT * SEG;        // [CIN][XW]
    const int D = a.d, H = a.h, W = a.w;
    const int64_t r0 = a.rows * s / a.S, r1 = a.rows * (s + 1) / a.S;
    const bool centre = (q == 4);

    f32x4 acc[C::CPW][3][C::IB];
#pragma unroll
    for (int i = 0; i < C::CPW; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < C::IB; ++k) acc[i][j][k] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;

    for (int64_t base = r0; base < r1; base += C::RS) {
        const int64_t r = base + rg;
        const int64_t t = r / H;
        const int yy = (int)(r - t * H), zz = (int)(t % D);
        const bool act = r < r1 && (unsigned)(zz + dz) < (unsigned)D && (unsigned)(yy + dy) < (unsigned)H;
        const int64_t src = r + (int64_t)dz * H + dy;  // source row index
        for (int x0 = 0; x0 < W; x0 += SEG) {
            __syncthreads();
            if (act) {
                // dy^T: 32 voxels x COUT channels, 8 channels per 16-byte
                // chunk.  Chunks go voxel fastest, so neighbouring lanes write
                // neighbouring LDS halves; channel fastest, the lanes of one
                // voxel wrote rows a multiple of 32 banks apart (8- and
                // 16-way bank conflicts: c5's weight gradient 0.120 -> 0.095 ms)
                for (int c = gt; c < SEG * COUT / 8; c += 64 * C::WS) {
                    const int j = c % SEG, c0 = (c / SEG) * 8;
                    uint4 v = {0u, 0u, 0u, 0u};
                    if (x0 + j < W) v = *reinterpret_cast<const uint4 *>(a.dy + ((r * W + x0 + j) * COUT + c0));
                    const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
                    for (int i = 0; i < 8; ++i) dyT[(c0 + i) * SEG + j] = e[i];
                }
                // x^T of the source row, xT[i][jj] = x[x0 + jj - 1][i] for
                // jj = 0 .. 33 (one copy; the three x shifts are taken from
                // it in registers below)
                for (int c = gt; c < (SEG + 2) * CIN / 8; c += 64 * C::WS) {
                    const int jj = c % (SEG + 2), c0 = (c / (SEG + 2)) * 8;
                    const int xg = x0 + jj - 1;
                    uint4 v = {0u, 0u, 0u, 0u};
                    if (xg >= 0 && xg < W) v = *reinterpret_cast<const uint4 *>(a.x + ((src * W + xg) * CIN + c0));
                    const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
                    for (int i = 0; i < 8; ++i) xT[(c0 + i) * C::XW + jj] = e[i];
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int cl = 0; cl < C::CPW; ++cl) {
                    const int co = (wi * C::CPW + cl) * 16 + r16;
                    const uint4 A = *reinterpret_cast<const uint4 *>(dyT + co * SEG + 8 * g);
#pragma unroll
                    for (int ib = 0; ib < C::IB; ++ib) {
                        // voxels 8g + dx .. 8g + dx + 7 of channel ib*16 + r16
                        // for dx = 0, 1, 2: two aligned reads, then shifts
                        // by 0, 1 and 2 bfloat16 elements
                        const uint16_t *row = xT + (ib * 16 + r16) * C::XW + 8 * g;
                        const uint4 L = *reinterpret_cast<const uint4 *>(row);
                        const uint4 R = *reinterpret_cast<const uint4 *>(row + 8);
                        const uint4 B1 = {(L.x >> 16) | (L.y << 16), (L.y >> 16) | (L.z << 16),
                                          (L.z >> 16) | (L.w << 16), (L.w >> 16) | (R.x << 16)};
                        const uint4 B2 = {L.y, L.z, L.w, R.x};
                        acc[cl][0][ib] = mfma16(A, L, acc[cl][0][ib]);
                        acc[cl][1][ib] = mfma16(A, B1, acc[cl][1][ib]);
                        acc[cl][2][ib] = mfma16(A, B2, acc[cl][2][ib]);
                    }
                }
                if (centre && gt < COUT) {
#pragma unroll 8
                    for (int j = 0; j < SEG; ++j) bacc += bf2f(dyT[gt * SEG + j]);
                }
            }
        }
    }
    // Partial sums of this (s, row group): lane holds o = cb*16 + 4g + e,
    // i = ib*16 + r16.
    const int64_t p = (int64_t)s * C::RS + rg;
    float *part = a.part + p * (int64_t)COUT * 27 * CIN;
#pragma unroll
    for (int cl = 0; cl < C::CPW; ++cl)
#pragma unroll
        for (int dxi = 0; dxi < 3; ++dxi)
#pragma unroll
            for (int ib = 0; ib < C::IB; ++ib)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int o = (wi * C::CPW + cl) * 16 + 4 * g + e;
                    const int tap = q * 3 + dxi;
                    part[((int64_t)o * 27 + tap) * CIN + ib * 16 + r16] = acc[cl][dxi][ib][e];
                }
    if (centre && gt < COUT) a.bpart[p * COUT + gt] = bacc;
}

// ---------------------------------------------------------------------------
// Weight gradient, ring-staged (input channels <= 64 on large grids).  One
// block of 9 wavefronts per job and 16 output channels (blockIdx.y); a job
// is (sample n, ZB output planes from z0, one 32-voxel x segment, a range of
// output rows y).  Wave q is the neighbour-row pair (dz, dy) = (q / 3 - 1,
// q % 3 - 1) and accumulates its three x taps.  The block marches y: each
// step stages dy^T of its ZB output rows and x^T of row y + 1 of the ZB + 2
// source planes into a three-row ring, so each x row segment is staged and
// read from memory once per job (ZB + 2 planes for ZB output planes)
// instead of once per (dz, dy) pair and output row, and each dy row once
// instead of nine times.  The MFMA operands and the x shifts are the direct
// kernel's.  Partial sums per job, added by the same fixed-order reduction.
// ---------------------------------------------------------------------------
template <int CIN, int ZB>
struct WrCfg {
    static constexpr int IB = CIN / 16;
    static constexpr int SEG = 32, XW = SEG + 8;
    static constexpr int NP = ZB + 2;                // source planes z0 - 1 .. z0 + ZB
    static constexpr int X_U16 = 3 * NP * CIN * XW;  // three-row ring of x^T
    static constexpr int D_U16 = ZB * 16 * SEG;       // dy^T of the output rows
    static constexpr int NT = 9 * 64;
};

struct WrArgs {
    const uint16_t *x;
    const uint16_t *dy;
    float *part;   // [jobs][COUT][27][CIN]
    float *bpart;  // [jobs][COUT]
    int d, h, w, cout;
    int nzb, nxs, ys;  // z blocks, x segments, y ranges per (n, z block, x segment)
};

template <int CIN, int ZB>
__global__ __launch_bounds__(576) __attribute__((amdgpu_waves_per_eu(CIN <= 16 ? 6 : CIN <= 32 ? 5 : 4, 8)))
void conv_wgrad_ring_kernel(WrArgs a)
{
    using C = WrCfg<CIN, ZB>;
    constexpr int SEG = C::SEG, XW = C::XW, NP = C::NP, IB = C::IB, NT = C::NT;
    __shared__ __attribute__((aligned(16))) uint16_t xr[C::X_U16];
    __shared__ __attribute__((aligned(16))) uint16_t dyT[C::D_U16];
    const int job = blockIdx.x, cb = blockIdx.y;
    const int tid = threadIdx.x, q = tid >> 6, lane = tid & 63;
    const int dz = q / 3 - 1, dq = q % 3 - 1;
    const int r16 = lane & 15, g = lane >> 4;
    int t = job;
    const int ysp = t % a.ys;
    t /= a.ys;
    const int xs = t % a.nxs;
    t /= a.nxs;
    const int zb = t % a.nzb, n = t / a.nzb;
    const int D = a.d, H = a.h, W = a.w, COUT = a.cout;
    const int z0 = zb * ZB, x0 = xs * SEG;
    const int ya = (int)((int64_t)H * ysp / a.ys), yb = (int)((int64_t)H * (ysp + 1) / a.ys);
    const int64_t nD = (int64_t)n * D;

    // x^T of source row yr of the NP planes, ring slot yr mod 3:
    // xr[slot][p][i][jj] = x[n][z0 - 1 + p][yr][x0 + jj - 1][i], jj = 0 .. 33.
    // Thread tid moves chunks tid, tid + NT, ... (8 channels of one voxel,
    // voxel fastest: neighbouring lanes write neighbouring LDS words); the
    // loads go to registers first, so that the next row's loads are in
    // flight while the current row's MFMAs run.
    constexpr int XCH = NP * (SEG + 2) * (CIN / 8), XPT = (XCH + NT - 1) / NT;
    constexpr int DCH = ZB * SEG * 2, DPT = (DCH + NT - 1) / NT;
    auto load_x = [&](int yr, uint4 (&v)[XPT]) {
#pragma unroll
        for (int k = 0; k < XPT; ++k) {
            const int c = tid + k * NT;
            const int jj = c % (SEG + 2), rest = c / (SEG + 2);
            const int c0 = (rest % (CIN / 8)) * 8, p = rest / (CIN / 8);
            const int zs = z0 - 1 + p, xg = x0 + jj - 1;
            v[k] = uint4{0u, 0u, 0u, 0u};
            if (c < XCH && (unsigned)yr < (unsigned)H && (unsigned)zs < (unsigned)D && (unsigned)xg < (unsigned)W)
                v[k] = *reinterpret_cast<const uint4 *>(a.x + ((((nD + zs) * H + yr) * W + xg) * CIN + c0));
        }
    };
    auto store_x = [&](int yr, const uint4 (&v)[XPT]) {
        const int slot = (yr + 3) % 3;
#pragma unroll
        for (int k = 0; k < XPT; ++k) {
            const int c = tid + k * NT;
            if (c >= XCH) break;
            const int jj = c % (SEG + 2), rest = c / (SEG + 2);
            const int c0 = (rest % (CIN / 8)) * 8, p = rest / (CIN / 8);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v[k]);
            uint16_t *dst = xr + ((slot * NP + p) * CIN + c0) * XW + jj;
#pragma unroll
            for (int i = 0; i < 8; ++i) dst[i * XW] = e[i];
        }
    };
    // dy^T of output rows (n, z0 + zi, y), channels cb*16 .. cb*16 + 15:
    // dyT[zi][o][j] = dy[n][z0 + zi][y][x0 + j][cb*16 + o]
    auto load_dy = [&](int y, uint4 (&v)[DPT]) {
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            const int c = tid + k * NT;
            const int j = c % SEG, rest = c / SEG;
            const int half = rest & 1, zi = rest >> 1;
            const int z = z0 + zi, xg = x0 + j;
            v[k] = uint4{0u, 0u, 0u, 0u};
            if (c < DCH && y < H && z < D && xg < W)
                v[k] = *reinterpret_cast<const uint4 *>(a.dy + ((((nD + z) * H + y) * W + xg) * COUT + cb * 16 + half * 8));
        }
    };
    auto store_dy = [&](const uint4 (&v)[DPT]) {
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            const int c = tid + k * NT;
            if (c >= DCH) break;
            const int j = c % SEG, rest = c / SEG;
            const int half = rest & 1, zi = rest >> 1;
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v[k]);
            uint16_t *dst = dyT + (zi * 16 + half * 8) * SEG + j;
#pragma unroll
            for (int i = 0; i < 8; ++i) dst[i * SEG] = e[i];
        }
    };

    f32x4 acc[3][IB];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < IB; ++k) acc[j][k] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;

    uint4 xv[XPT], dv[DPT];
    for (int yr = ya - 1; yr <= ya + 1; ++yr) {
        load_x(yr, xv);
        store_x(yr, xv);
    }
    load_dy(ya, dv);
    store_dy(dv);
    __syncthreads();
    for (int y = ya; y < yb; ++y) {
        // next step's rows (x row y + 2, dy row y + 1) in flight during this step
        const bool more = y + 1 < yb;
        if (more) {
            load_x(y + 2, xv);
            load_dy(y + 1, dv);
        }
        const int sy = y + dq;
        if ((unsigned)sy < (unsigned)H) {
            const uint16_t *xs_row = xr + ((sy % 3) * NP + 1 + dz) * CIN * XW;
#pragma unroll
            for (int zi = 0; zi < ZB; ++zi) {
                const uint4 A = *reinterpret_cast<const uint4 *>(dyT + (zi * 16 + r16) * SEG + 8 * g);
#pragma unroll
                for (int ib = 0; ib < IB; ++ib) {
                    // voxels 8g + dx .. 8g + dx + 7 of channel ib*16 + r16 of
                    // plane z0 + zi + dz, for dx = 0, 1, 2
                    const uint16_t *row = xs_row + (zi * CIN + ib * 16 + r16) * XW + 8 * g;
                    const uint4 L = *reinterpret_cast<const uint4 *>(row);
                    const uint4 R = *reinterpret_cast<const uint4 *>(row + 8);
                    const uint4 B1 = {(L.x >> 16) | (L.y << 16), (L.y >> 16) | (L.z << 16),
                                      (L.z >> 16) | (L.w << 16), (L.w >> 16) | (R.x << 16)};
                    const uint4 B2 = {L.y, L.z, L.w, R.x};
                    acc[0][ib] = mfma16(A, L, acc[0][ib]);
                    acc[1][ib] = mfma16(A, B1, acc[1][ib]);
                    acc[2][ib] = mfma16(A, B2, acc[2][ib]);
                }
            }
        }
        if (q == 4) {  // bias: lane (o = r16, g) sums voxels 8g .. 8g + 7 of every output row
#pragma unroll
            for (int zi = 0; zi < ZB; ++zi)
#pragma unroll
                for (int j = 0; j < 8; ++j) bacc += bf2f(dyT[(zi * 16 + r16) * SEG + 8 * g + j]);
        }
        __syncthreads();  // every wave is done with dy^T and ring slot (y - 1) mod 3 = (y + 2) mod 3
        if (more) {
            store_x(y + 2, xv);
            store_dy(dv);
        }
        __syncthreads();
    }
    // Partial sums of this job: lane holds o = cb*16 + 4g + e, i = ib*16 + r16.
    float *part = a.part + (int64_t)job * COUT * 27 * CIN;
#pragma unroll
    for (int dxi = 0; dxi < 3; ++dxi)
#pragma unroll
        for (int ib = 0; ib < IB; ++ib)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = cb * 16 + 4 * g + e;
                part[((int64_t)o * 27 + q * 3 + dxi) * CIN + ib * 16 + r16] = acc[dxi][ib][e];
            }
    if (q == 4) {  // the four voxel groups of each channel, added in a fixed order
        const float b1 = __shfl_down(bacc, 16), b2 = __shfl_down(bacc, 32), b3 = __shfl_down(bacc, 48);
        if (lane < 16) a.bpart[(int64_t)job * COUT + cb * 16 + lane] = (bacc + b1) + (b2 + b3);
    }
}

// Fixed-order sum of P partial arrays: out[c][i] = sum of partials
// c*chunk .. min(P, (c+1)*chunk) - 1 in increasing order (blockIdx.y = c).
// Two passes (chunks, then the chunk sums) give the same result on every
// run.  One launch per pass covers two arrays (the weights, n0 floats per
// partial, then the biases, n1), each summed on its own.
// Partials per chunk of the first pass: 32, or 128 from 2048 partials on
// (the one-channel layers at 128^3 have 8192: 32 per chunk left 256 chunk
// sums for the second pass, a chain of dependent loads per thread).
constexpr int64_t kSumChunk = 32, kSumChunkLarge = 128, kSumLargeFrom = 2048;
inline int64_t sum_chunk(int64_t P) { return P >= kSumLargeFrom ? kSumChunkLarge : kSumChunk; }

struct SumSet {
    const float *part;
    float *out;
    int64_t n;
};

// One 256-thread block of the reduction: block column bx, chunk row by.
__device__ __forceinline__ void sum_parts_block(const SumSet &s0, const SumSet &s1, int64_t P, int chunk,
                                                int64_t bx, int64_t by)
{
    int64_t i = bx * blockDim.x + threadIdx.x;
    const bool first = i < s0.n;
    if (!first) i -= s0.n;
    const SumSet &S = first ? s0 : s1;
    if (i >= S.n) return;
    const int64_t n = S.n;
    const float *part = S.part;
    const int64_t p0 = by * chunk;
    const int64_t p1 = p0 + chunk < P ? p0 + chunk : P;
    // eight loads in flight, then added in the same increasing order
    float s = 0.f;
    int64_t p = p0;
    for (; p + 8 <= p1; p += 8) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = part[(p + k) * n + i];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; p < p1; ++p) s += part[p * n + i];
    S.out[by * n + i] = s;
}

__global__ void sum_parts_kernel(SumSet s0, SumSet s1, int64_t P, int chunk)
{
    sum_parts_block(s0, s1, P, chunk, blockIdx.x, blockIdx.y);
}

// Several layers' reductions in one launch: layer k owns the flat block
// range [start[k], start[k+1]), laid out as rows of bx[k] blocks, one row per
// chunk.  Each block does what sum_parts_kernel's block (column, row) does
// for that layer, so the sums are the same bits.
struct SumMany {
    SumSet w[UNET_WGRAD_MAX], b[UNET_WGRAD_MAX];
    int64_t P[UNET_WGRAD_MAX];
    int32_t chunk[UNET_WGRAD_MAX], bx[UNET_WGRAD_MAX];
    int64_t start[UNET_WGRAD_MAX + 1];
    int32_t count;
};

__global__ void sum_parts_many_kernel(SumMany m)
{
    const int64_t f = blockIdx.x;
    int k = 0;
    while (k + 1 < m.count && f >= m.start[k + 1]) ++k;
    const int64_t local = f - m.start[k];
    sum_parts_block(m.w[k], m.b[k], m.P[k], m.chunk[k], local % m.bx[k], local / m.bx[k]);
}

// Sums P partials of n0 and of n1 floats (n1 may be 0) through tmp0 / tmp1
// (Q = ceil(P / chunk) chunk sums each) into out0 / out1.
hipError_t sum_parts(const float *part0, int64_t n0, float *tmp0, float *out0, const float *part1, int64_t n1,
                     float *tmp1, float *out1, int64_t P, hipStream_t st)
{
    const int64_t C = sum_chunk(P), Q = (P + C - 1) / C;
    const unsigned bx = (unsigned)((n0 + n1 + 255) / 256);
    hipLaunchKernelGGL(sum_parts_kernel, dim3(bx, (unsigned)Q), dim3(256), 0, st, SumSet{part0, tmp0, n0},
                       SumSet{part1, tmp1, n1}, P, (int)C);
    hipLaunchKernelGGL(sum_parts_kernel, dim3(bx, 1), dim3(256), 0, st, SumSet{tmp0, out0, n0},
                       SumSet{tmp1, out1, n1}, Q, (int)Q);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One-channel layers (the network's input and output): a 1 -> 16 or 16 -> 1
// convolution is 432 multiply-adds per voxel, too thin for the matrix
// cores, so one thread computes one voxel on the vector units.  Weights
// (bfloat16, the packed layout [COUT][27][CIN]) are held in LDS as floats.
// ---------------------------------------------------------------------------
constexpr int kThin = 16;  // channels on the wide side

__device__ __forceinline__ void thin_decode(int64_t v, int D, int H, int W, int &z, int &y, int &x)
{
    if (v <= 0xffffffffll) {  // 32-bit division, far cheaper than the 64-bit sequence
        const uint32_t u = (uint32_t)v, t = u / (uint32_t)W, t2 = t / (uint32_t)H;
        x = (int)(u - t * (uint32_t)W);
        y = (int)(t - t2 * (uint32_t)H);
        z = (int)(t2 % (uint32_t)D);
        return;
    }
    const int64_t t = v / W;
    x = (int)(v - t * W);
    const int64_t t2 = t / H;
    y = (int)(t - t2 * H);
    z = (int)(t2 % D);
}

__device__ __forceinline__ bool thin_tap(int tap, int z, int y, int x, int D, int H, int W, int64_t HW,
                                         int64_t &off)
{
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    off = dz * HW + (int64_t)dy * W + dx;
    return (unsigned)(z + dz) < (unsigned)D && (unsigned)(y + dy) < (unsigned)H && (unsigned)(x + dx) < (unsigned)W;
}

// The fused epilogue of conv_fwd_kernel for one voxel and channel.
__device__ __forceinline__ void thin_store(const ConvArgs &a, int64_t v, int co, int cout, float acc)
{
    float val = acc + (a.bias ? a.bias[co] : 0.f);
    if (a.relu) val = fmaxf(val, 0.f);
    if (a.y && co < a.ych) a.y[v * a.ych + co] = val;
    const int64_t o = v * cout + co;
    if (a.r) a.r[o] = f2bf(val);
    if (a.out) a.out[o] = f2bf(a.skip ? val + bf2f(a.skip[o]) : val);
}

// 1 -> 16 channels.  Weights in LDS as [tap][channel] so that one tap's
// sixteen weights are four 16-byte reads; each channel sums its taps in
// ascending order.
__global__ __launch_bounds__(256) void conv_thin_in_kernel(ConvArgs a)
{
    __shared__ float4 wsh4[27 * kThin / 4];
    float *wsh = reinterpret_cast<float *>(wsh4);
    for (int i = threadIdx.x; i < kThin * 27; i += blockDim.x) wsh[(i % 27) * kThin + i / 27] = bf2f(a.wt[i]);
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t vbase = v - lane;  // the wavefront's first voxel
    // whole wavefronts only: the stores at the end are shared by its lanes
    if (vbase >= a.nvox) return;
    const bool live = v < a.nvox;
    int z, y, x;
    thin_decode(live ? v : vbase, a.d, a.h, a.w, z, y, x);
    const int64_t HW = (int64_t)a.h * a.w;
    float acc[kThin];
#pragma unroll
    for (int co = 0; co < kThin; ++co) acc[co] = 0.f;
#pragma unroll 3
    for (int t = 0; t < 27; ++t) {
        int64_t off;
        const float xt = thin_tap(t, z, y, x, a.d, a.h, a.w, HW, off) && live ? bf2f(a.x[v + off]) : 0.f;
#pragma unroll
        for (int q = 0; q < kThin / 4; ++q) {
            const float4 w4 = wsh4[t * (kThin / 4) + q];
            acc[4 * q] = fmaf(w4.x, xt, acc[4 * q]);
            acc[4 * q + 1] = fmaf(w4.y, xt, acc[4 * q + 1]);
            acc[4 * q + 2] = fmaf(w4.z, xt, acc[4 * q + 2]);
            acc[4 * q + 3] = fmaf(w4.w, xt, acc[4 * q + 3]);
        }
    }
    float val[kThin];
#pragma unroll
    for (int co = 0; co < kThin; ++co) {
        const float t = acc[co] + (a.bias ? a.bias[co] : 0.f);
        val[co] = a.relu ? fmaxf(t, 0.f) : t;
    }
    // The epilogue of thin_store for all 16 channels.  Each output goes
    // through the wavefront's LDS rows (voxel lane, kEpiStride floats) so
    // that a store instruction writes 1 KB contiguous across the lanes
    // instead of 16 bytes per lane at a 32- or 64-byte stride.
    __shared__ __attribute__((aligned(16))) float tscr[4][64 * kEpiStride];
    float *scr = tscr[threadIdx.x >> 6];
    const int nlive = (int)(a.nvox - vbase < 64 ? a.nvox - vbase : 64);
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // 16 bfloat16 (two 16-byte chunks) per voxel
    auto store_bf16 = [&](uint16_t *dst, const uint32_t (&w)[kThin / 2]) {
        uint4 *row = reinterpret_cast<uint4 *>(scr + lane * kEpiStride);
        row[0] = make_uint4(w[0], w[1], w[2], w[3]);
        row[1] = make_uint4(w[4], w[5], w[6], w[7]);
        wave_sync();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int chunk = k * 64 + lane, vox = chunk >> 1;
            if (vox < nlive)
                *reinterpret_cast<uint4 *>(dst + vbase * kThin + chunk * 8) =
                    *reinterpret_cast<const uint4 *>(scr + vox * kEpiStride + 4 * (chunk & 1));
        }
        wave_sync();  // reads done before the rows are written again
    };
    if (a.y) {
        if (a.ych == kThin) {
            float4 *row = reinterpret_cast<float4 *>(scr + lane * kEpiStride);
#pragma unroll
            for (int q = 0; q < 4; ++q) row[q] = make_float4(val[4 * q], val[4 * q + 1], val[4 * q + 2], val[4 * q + 3]);
            wave_sync();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int chunk = k * 64 + lane, vox = chunk >> 2;
                if (vox < nlive)
                    *reinterpret_cast<float4 *>(a.y + vbase * kThin + chunk * 4) =
                        *reinterpret_cast<const float4 *>(scr + vox * kEpiStride + 4 * (chunk & 3));
            }
            wave_sync();
        } else if (live) {
#pragma unroll
            for (int co = 0; co < kThin; ++co)
                if (co < a.ych) a.y[v * a.ych + co] = val[co];
        }
    }
    uint32_t rb[kThin / 2], ob[kThin / 2];
#pragma unroll
    for (int q = 0; q < kThin / 2; ++q) {
        rb[q] = (uint32_t)f2bf(val[2 * q]) | ((uint32_t)f2bf(val[2 * q + 1]) << 16);
        if (a.out) {
            float o0 = val[2 * q], o1 = val[2 * q + 1];
            if (a.skip && live) {
                o0 += bf2f(a.skip[v * kThin + 2 * q]);
                o1 += bf2f(a.skip[v * kThin + 2 * q + 1]);
            }
            ob[q] = (uint32_t)f2bf(o0) | ((uint32_t)f2bf(o1) << 16);
        }
    }
    if (a.r) store_bf16(a.r, rb);
    if (a.gout) {  // the next layer's ReLU gradient
        uint4 m0 = make_uint4(0u, 0u, 0u, 0u), m1 = m0;
        if (live) {
            const uint4 *pm = reinterpret_cast<const uint4 *>(a.mask + v * kThin);
            m0 = pm[0];
            m1 = pm[1];
        }
        const uint16_t *me0 = reinterpret_cast<const uint16_t *>(&m0);
        const uint16_t *me1 = reinterpret_cast<const uint16_t *>(&m1);
        uint32_t gb[kThin / 2];
#pragma unroll
        for (int q = 0; q < kThin / 2; ++q) {
            const uint16_t *me = q < 4 ? me0 : me1;
            const int k = (2 * q) & 7;
            gb[q] = (uint32_t)(bf2f(me[k]) > 0.f ? f2bf(val[2 * q]) : (uint16_t)0) |
                    ((uint32_t)(bf2f(me[k + 1]) > 0.f ? f2bf(val[2 * q + 1]) : (uint16_t)0) << 16);
        }
        store_bf16(a.gout, gb);
    }
    if (a.out) store_bf16(a.out, ob);
}

// 16 -> 1 channel.
__global__ __launch_bounds__(256) void conv_thin_out_kernel(ConvArgs a)
{
    __shared__ float wsh[27 * kThin];
    for (int i = threadIdx.x; i < 27 * kThin; i += blockDim.x) wsh[i] = bf2f(a.wt[i]);
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.nvox) return;
    int z, y, x;
    thin_decode(v, a.d, a.h, a.w, z, y, x);
    const int64_t HW = (int64_t)a.h * a.w;
    float acc = 0.f;
    for (int t = 0; t < 27; ++t) {
        int64_t off;
        if (!thin_tap(t, z, y, x, a.d, a.h, a.w, HW, off)) continue;
        const uint4 *p = reinterpret_cast<const uint4 *>(a.x + (v + off) * kThin);
        const uint4 c0 = p[0], c1 = p[1];
        const uint16_t *e0 = reinterpret_cast<const uint16_t *>(&c0);
        const uint16_t *e1 = reinterpret_cast<const uint16_t *>(&c1);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc = fmaf(wsh[t * kThin + i], bf2f(e0[i]), acc);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc = fmaf(wsh[t * kThin + 8 + i], bf2f(e1[i]), acc);
    }
    thin_store(a, v, 0, 1, acc);
}

// ---------------------------------------------------------------------------
// Weight gradient of the one-channel layers on the matrix cores.  With W the
// 16-channel operand (dy of the 1 -> 16 layer, x of the 16 -> 1 layer) and
// T the one-channel one (x, resp. dy), the MFMA takes A = W^T [16 channels]
// [32 voxels of an output row segment] and B[k][t] = T at voxel k moved by
// tap t = (dz, dy, dx) (27 taps in two 16-column tiles), so that
// C[c][t] = sum_k W[k][c] T[k + off(t)].  For 1 -> 16 that is dw[c][t]; for
// 16 -> 1, dw[t][c] = sum_u x[u][c] dy[u - off(t)] is C[c][26 - t].  A job
// is (n, 4 planes, a 32-voxel x segment, a y range) as in the ring kernel;
// wave w of the block takes output plane z0 + w, the block marches y with a
// three-row ring of T rows of the 6 planes z0 - 1 .. z0 + 4 (x^T of the
// voxels x0 - 1 .. x0 + 32), and each wave writes its own partial sums.
// ---------------------------------------------------------------------------
constexpr int kThinZB = 4, kThinSeg = 32, kThinXW = kThinSeg + 8, kThinNP = kThinZB + 2;

struct WtArgs {
    const uint16_t *w16;  // the 16-channel operand, channels-last
    const uint16_t *t1;   // the one-channel operand
    float *part;          // [jobs * 4][432]
    float *bpart;         // [jobs * 4][16 or 1]
    int d, h, w;
    int nzb, nxs, ys;
};

template <bool IN1>
__global__ __launch_bounds__(256) void wgrad_thin_mfma_kernel(WtArgs a)
{
    constexpr int SEG = kThinSeg, XW = kThinXW, NP = kThinNP, ZB = kThinZB, C16 = kThin;
    __shared__ __attribute__((aligned(16))) uint16_t tr[3 * NP * XW];       // ring of T rows
    __shared__ __attribute__((aligned(16))) uint16_t wT[ZB * C16 * SEG];    // W^T of the output rows
    const int job = blockIdx.x, tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, g = lane >> 4;
    int t = job;
    const int ysp = t % a.ys;
    t /= a.ys;
    const int xs = t % a.nxs;
    t /= a.nxs;
    const int zb = t % a.nzb, n = t / a.nzb;
    const int D = a.d, H = a.h, W = a.w;
    const int z0 = zb * ZB, x0 = xs * SEG;
    const int ya = (int)((int64_t)H * ysp / a.ys), yb = (int)((int64_t)H * (ysp + 1) / a.ys);
    const int64_t nD = (int64_t)n * D;

    // T row yr of the NP planes into ring slot yr mod 3: tr[slot][p][jj] =
    // T[n][z0 - 1 + p][yr][x0 + jj - 1], jj = 0 .. 33 (one value per thread)
    auto stage_t = [&](int yr) {
        const int slot = (yr + 3) % 3;
        for (int c = tid; c < NP * (SEG + 2); c += 256) {
            const int jj = c % (SEG + 2), p = c / (SEG + 2);
            const int zs = z0 - 1 + p, xg = x0 + jj - 1;
            uint16_t v = 0;
            if ((unsigned)yr < (unsigned)H && (unsigned)zs < (unsigned)D && (unsigned)xg < (unsigned)W)
                v = a.t1[((nD + zs) * H + yr) * W + xg];
            tr[(slot * NP + p) * XW + jj] = v;
        }
    };
    // W^T of output rows (n, z0 + zi, y): wT[zi][c][j] = W[n][z0 + zi][y][x0 + j][c]
    auto stage_w = [&](int y) {
        for (int c = tid; c < ZB * SEG * 2; c += 256) {
            const int j = c % SEG, rest = c / SEG;
            const int half = rest & 1, zi = rest >> 1;
            const int z = z0 + zi, xg = x0 + j;
            uint4 v = {0u, 0u, 0u, 0u};
            if (z < D && xg < W)
                v = *reinterpret_cast<const uint4 *>(a.w16 + (((nD + z) * H + y) * W + xg) * C16 + half * 8);
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
            uint16_t *dst = wT + (zi * C16 + half * 8) * SEG + j;
#pragma unroll
            for (int i = 0; i < 8; ++i) dst[i * SEG] = e[i];
        }
    };

    // this lane's taps in the two column tiles: t = tt * 16 + r16
    int tdz[2], tdy[2], tsh[2];
    bool tok[2];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        const int tap = tt * 16 + r16;
        tok[tt] = tap < 27;
        tdz[tt] = tap / 9 - 1;
        tdy[tt] = (tap / 3) % 3 - 1;
        tsh[tt] = tap % 3;  // jj shift: voxel x0 + k + dx sits at jj = k + dx + 1
    }
    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    float bacc = 0.f;

    stage_t(ya - 1);
    stage_t(ya);
    for (int y = ya; y < yb; ++y) {
        stage_t(y + 1);
        stage_w(y);
        __syncthreads();
        const uint4 A = *reinterpret_cast<const uint4 *>(wT + (wv * C16 + r16) * SEG + 8 * g);
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            uint4 B = {0u, 0u, 0u, 0u};
            const int sy = y + tdy[tt];
            if (tok[tt] && (unsigned)sy < (unsigned)H) {
                const uint16_t *row = tr + ((sy % 3) * NP + wv + 1 + tdz[tt]) * XW + 8 * g;
                const uint4 L = *reinterpret_cast<const uint4 *>(row);
                const uint4 R = *reinterpret_cast<const uint4 *>(row + 8);
                const uint4 B1 = {(L.x >> 16) | (L.y << 16), (L.y >> 16) | (L.z << 16),
                                  (L.z >> 16) | (L.w << 16), (L.w >> 16) | (R.x << 16)};
                const uint4 B2 = {L.y, L.z, L.w, R.x};
                B = tsh[tt] == 0 ? L : (tsh[tt] == 1 ? B1 : B2);
            }
            acc[tt] = mfma16(A, B, acc[tt]);
        }
        if (IN1) {  // bias of the 16 channels: lane (c = r16, g) sums voxels 8g .. 8g + 7
#pragma unroll
            for (int j = 0; j < 8; ++j) bacc += bf2f(wT[(wv * C16 + r16) * SEG + 8 * g + j]);
        } else if (lane < SEG) {  // bias of the one channel: dy of this output row, one voxel per lane
            bacc += bf2f(tr[((y % 3) * NP + wv + 1) * XW + lane + 1]);
        }
        __syncthreads();  // every wave is done with this step's ring slot and W^T
    }
    // partial sums of (job, wave): lane holds c = 4g + e, t = tt*16 + r16
    const int64_t pw = (int64_t)job * ZB + wv;
    float *part = a.part + pw * 27 * C16;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        if (!tok[tt]) continue;
        const int tap = tt * 16 + r16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 4 * g + e;
            // (1, 16): dw[c][tap][0]; (16, 1): dw[0][26 - tap][c]
            part[IN1 ? c * 27 + tap : (26 - tap) * C16 + c] = acc[tt][e];
        }
    }
    if (IN1) {  // the four voxel groups of each channel, in a fixed order
        const float b1 = __shfl_down(bacc, 16), b2 = __shfl_down(bacc, 32), b3 = __shfl_down(bacc, 48);
        if (lane < 16) a.bpart[pw * C16 + lane] = (bacc + b1) + (b2 + b3);
    } else {  // fixed butterfly over the lanes
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) bacc += __shfl_xor(bacc, m, 64);
        if (lane == 0) a.bpart[pw] = bacc;
    }
}


// ---------------------------------------------------------------------------
// Element-wise and resampling kernels
// ---------------------------------------------------------------------------
__global__ void weight_pack_kernel(const float *__restrict__ w, int cin, int cout, uint16_t *__restrict__ wf,
                                   uint16_t *__restrict__ wb)
{
    const int64_t n = (int64_t)cout * 27 * cin;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = (int)(i % cin);
    const int t = (int)((i / cin) % 27);
    const int co = (int)(i / (27 * (int64_t)cin));
    const uint16_t b = f2bf(w[i]);
    if (wf) wf[i] = b;
    if (wb) wb[(int64_t)ci * 27 * cout + (int64_t)(26 - t) * cout + co] = b;
}

// weight_pack_kernel over several layers: element i of the concatenation
// of their weights (start[k] the first element of layer k).
struct PackSet {
    unet_pack_item_t item[UNET_PACK_MAX];
    int64_t start[UNET_PACK_MAX + 1];
    int count;
};

// SMALL: every layer has fewer than 2^32 weights, so the index is split in
// 32-bit arithmetic (the 64-bit divisions are emulated in software).
template <bool SMALL>
__global__ void weight_pack_many_kernel(PackSet P)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.start[P.count]) return;
    int k = 0;
    while (i >= P.start[k + 1]) ++k;
    const unet_pack_item_t &L = P.item[k];
    const int64_t j = i - P.start[k];
    int ci, t, co;
    if constexpr (SMALL) {
        const uint32_t j32 = (uint32_t)j, jt = j32 / (uint32_t)L.cin;
        ci = (int)(j32 - jt * (uint32_t)L.cin);
        t = (int)(jt % 27u);
        co = (int)(jt / 27u);
    } else {
        ci = (int)(j % L.cin);
        t = (int)((j / L.cin) % 27);
        co = (int)(j / (27 * (int64_t)L.cin));
    }
    const uint16_t b = f2bf(L.w[j]);
    if (L.w_fwd) L.w_fwd[j] = b;
    if (L.w_bwd) L.w_bwd[(int64_t)ci * 27 * L.cout + (int64_t)(26 - t) * L.cout + co] = b;
}

__global__ void embed_kernel(int64_t nvox, int ch, const float *__restrict__ img, float scale,
                             uint16_t *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nvox * ch) return;
    const int64_t v = i / ch;
    x[i] = (i - v * ch) == 0 ? f2bf(img[v] * scale) : (uint16_t)0;
}

// embed_kernel for eight consecutive elements per thread, stored as one
// 16-byte vector (the element count a multiple of 8, x 16-byte aligned).
__global__ void embed8_kernel(int64_t nvox, int ch, const float *__restrict__ img, float scale,
                              uint16_t *__restrict__ x)
{
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
    if (i0 >= nvox * ch) return;
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t h[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t i = i0 + 2 * q + e;
            if (ch == 1) {
                h[e] = f2bf(img[i] * scale);
            } else {
                const int64_t v = i / ch;
                h[e] = (i - v * ch) == 0 ? f2bf(img[v] * scale) : 0u;
            }
        }
        w[q] = h[0] | (h[1] << 16);
    }
    *reinterpret_cast<uint4 *>(x + i0) = make_uint4(w[0], w[1], w[2], w[3]);
}

// Index i of an [n][d][h][w][cg] array as (g, x, y, z, n), in 32-bit
// arithmetic when the array has fewer than 2^32 elements.
__device__ __forceinline__ void decode5(int64_t i, int64_t total, int cg, int w, int h, int d, int &g, int &x, int &y,
                                        int &z, int64_t &nn)
{
    if (total <= 0xffffffffll) {
        uint32_t t = (uint32_t)i;
        g = (int)(t % (uint32_t)cg);
        t /= (uint32_t)cg;
        x = (int)(t % (uint32_t)w);
        t /= (uint32_t)w;
        y = (int)(t % (uint32_t)h);
        t /= (uint32_t)h;
        z = (int)(t % (uint32_t)d);
        nn = t / (uint32_t)d;
    } else {
        int64_t t = i;
        g = (int)(t % cg);
        t /= cg;
        x = (int)(t % w);
        t /= w;
        y = (int)(t % h);
        t /= h;
        z = (int)(t % d);
        nn = t / d;
    }
}

// One thread per (coarse voxel, 8-channel group).
__global__ void pool2_kernel(int n, int d, int h, int w, int c, const uint16_t *__restrict__ x,
                             uint16_t *__restrict__ y)
{
    const int d2 = d / 2, h2 = h / 2, w2 = w / 2, cg = c / 8;
    const int64_t total = (int64_t)n * d2 * h2 * w2 * cg;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int gi, xo, yo, zo;
    int64_t nn;
    decode5(i, total, cg, w2, h2, d2, gi, xo, yo, zo, nn);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 8; ++k) {
        const int64_t v = ((nn * d + 2 * zo + (k >> 2)) * h + 2 * yo + ((k >> 1) & 1)) * w + 2 * xo + (k & 1);
        const uint4 q = *reinterpret_cast<const uint4 *>(x + v * c + gi * 8);
        const uint16_t *e = reinterpret_cast<const uint16_t *>(&q);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += bf2f(e[j]);
    }
    uint4 o;
    uint16_t *oe = reinterpret_cast<uint16_t *>(&o);
#pragma unroll
    for (int j = 0; j < 8; ++j) oe[j] = f2bf(s[j] * 0.125f);
    const int64_t vo = ((nn * d2 + zo) * h2 + yo) * w2 + xo;
    *reinterpret_cast<uint4 *>(y + vo * c + gi * 8) = o;
}

// One thread per (fine voxel, 8-channel group): nearest-neighbour copy.
__global__ void up2_kernel(int n, int d, int h, int w, int c, const uint16_t *__restrict__ x,
                           uint16_t *__restrict__ y)
{
    const int D = 2 * d, H = 2 * h, W = 2 * w, cg = c / 8;
    const int64_t total = (int64_t)n * D * H * W * cg;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int gi, xf, yf, zf;
    int64_t nn;
    decode5(i, total, cg, W, H, D, gi, xf, yf, zf, nn);
    const int64_t vc = ((nn * d + zf / 2) * h + yf / 2) * w + xf / 2;
    const int64_t vf = ((nn * D + zf) * H + yf) * W + xf;
    *reinterpret_cast<uint4 *>(y + vf * c + gi * 8) = *reinterpret_cast<const uint4 *>(x + vc * c + gi * 8);
}

// out[e] = g[e] where mask[e] > 0, else 0, in bfloat16, for VEC consecutive
// elements; VEC = 4 reads the mask and writes out as one 8-byte access each
// (both 8-byte aligned: the launch checks the base pointers).
template <int VEC>
__device__ __forceinline__ void relu_mask_store(const uint16_t *mask, const float (&g)[VEC], uint16_t *out)
{
    if constexpr (VEC == 4) {
        const uint2 m = *reinterpret_cast<const uint2 *>(mask);
        const uint16_t mk[4] = {(uint16_t)(m.x & 0xffffu), (uint16_t)(m.x >> 16), (uint16_t)(m.y & 0xffffu),
                                (uint16_t)(m.y >> 16)};
        uint32_t o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = bf2f(mk[e]) > 0.f ? f2bf(g[e]) : 0u;
        *reinterpret_cast<uint2 *>(out) = uint2{o[0] | (o[1] << 16), o[2] | (o[3] << 16)};
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) out[e] = bf2f(mask[e]) > 0.f ? f2bf(g[e]) : (uint16_t)0;
    }
}

// One thread per (coarse voxel, VEC consecutive channels): each channel's sum
// of the 8 children in a fixed order; the index is decoded once, in 32-bit
// arithmetic when it fits.
template <int VEC>
__global__ void up2_bwd_kernel(int n, int d, int h, int w, int c, const float *__restrict__ gf,
                               float *__restrict__ gc, const uint16_t *__restrict__ mask, uint16_t *__restrict__ gout)
{
    const int64_t total = (int64_t)n * d * h * w * c;
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
    if (i0 >= total) return;
    int ch, xc, yc, zc;
    int64_t nn;
    decode5(i0, total, c, w, h, d, ch, xc, yc, zc, nn);
    const int D = 2 * d, H = 2 * h, W = 2 * w;
    float s[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) s[e] = 0.f;
    for (int k = 0; k < 8; ++k) {
        const int64_t v = ((nn * D + 2 * zc + (k >> 2)) * H + 2 * yc + ((k >> 1) & 1)) * W + 2 * xc + (k & 1);
#pragma unroll
        for (int e = 0; e < VEC; ++e) s[e] += gf[v * c + ch + e];
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) gc[i0 + e] = s[e];
    if (gout)  // the ReLU gradient of the coarse level
        relu_mask_store<VEC>(mask + i0, s, gout + i0);
}

// VEC consecutive channels of one voxel per thread (VEC divides c); the
// fine-to-coarse index is decoded once, in 32-bit arithmetic when it fits.
template <int VEC>
__global__ void relu_grad_kernel(int n, int d, int h, int w, int c, const float *__restrict__ g1,
                                 const float *__restrict__ g2, const float *__restrict__ gp,
                                 const uint16_t *__restrict__ mask, uint16_t *__restrict__ out)
{
    const int64_t total = (int64_t)n * d * h * w * c;
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
    if (i0 >= total) return;
    float g[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) g[e] = g1[i0 + e];
    if (g2)
#pragma unroll
        for (int e = 0; e < VEC; ++e) g[e] += g2[i0 + e];
    if (gp) {
        int ch, xf, yf, zf;
        int64_t nn;
        if (total <= 0xffffffffll) {
            uint32_t t = (uint32_t)i0;
            ch = (int)(t % (uint32_t)c);
            t /= (uint32_t)c;
            xf = (int)(t % (uint32_t)w);
            t /= (uint32_t)w;
            yf = (int)(t % (uint32_t)h);
            t /= (uint32_t)h;
            zf = (int)(t % (uint32_t)d);
            nn = t / (uint32_t)d;
        } else {
            int64_t t = i0;
            ch = (int)(t % c);
            t /= c;
            xf = (int)(t % w);
            t /= w;
            yf = (int)(t % h);
            t /= h;
            zf = (int)(t % d);
            nn = t / d;
        }
        const int64_t vc = ((nn * (d / 2) + zf / 2) * (h / 2) + yf / 2) * (w / 2) + xf / 2;
#pragma unroll
        for (int e = 0; e < VEC; ++e) g[e] += gp[vc * c + ch + e] * 0.125f;
    }
    relu_mask_store<VEC>(mask + i0, g, out + i0);
}

constexpr int kMseBlocks = 1024;

__global__ void mse_kernel(int64_t nvox, int ch, const float *__restrict__ img, const float *__restrict__ y,
                           const float *__restrict__ tgt, float *__restrict__ out, uint16_t *__restrict__ gy,
                           double *__restrict__ part)
{
    __shared__ double red[256];
    double s = 0.0;
    const float gscale = 2.0f / (float)nvox;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * blockDim.x) {
        const float o = img[v] + y[v];
        if (out) out[v] = o;
        if (tgt) {
            const float df = o - tgt[v];
            s += (double)df * (double)df;
            if (gy) {
                gy[v * ch] = f2bf(gscale * df);
                for (int k = 1; k < ch; ++k) gy[v * ch + k] = 0;
            }
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// mse_kernel for one channel, four voxels per step: 16-byte loads of img, y
// and tgt, a 16-byte store of out and an 8-byte store of gy (nvox a multiple
// of 4; the launch checks the alignments).  out and gy get the same bits;
// the loss sums the same squares in another order.
__global__ void mse4_kernel(int64_t nvox, const float *__restrict__ img, const float *__restrict__ y,
                            const float *__restrict__ tgt, float *__restrict__ out, uint16_t *__restrict__ gy,
                            double *__restrict__ part)
{
    __shared__ double red[256];
    double s = 0.0;
    const float gscale = 2.0f / (float)nvox;
    const int64_t n4 = nvox / 4;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += (int64_t)gridDim.x * blockDim.x) {
        const float4 a = reinterpret_cast<const float4 *>(img)[q], b = reinterpret_cast<const float4 *>(y)[q];
        const float o[4] = {a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w};
        if (out) reinterpret_cast<float4 *>(out)[q] = make_float4(o[0], o[1], o[2], o[3]);
        if (tgt) {
            const float4 t = reinterpret_cast<const float4 *>(tgt)[q];
            const float df[4] = {o[0] - t.x, o[1] - t.y, o[2] - t.z, o[3] - t.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) s += (double)df[e] * (double)df[e];
            if (gy) {
                uint32_t g[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) g[e] = f2bf(gscale * df[e]);
                reinterpret_cast<uint2 *>(gy)[q] = uint2{g[0] | (g[1] << 16), g[2] | (g[3] << 16)};
            }
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void mse_final_kernel(const double *__restrict__ part, int nparts, int64_t nvox, double *__restrict__ loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (double)nvox;
}

__global__ void adam_kernel(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float omb1, float omb2, float eps,
                            float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int bad(const char *msg) { return rtm::set_error(RTM_EINVAL, msg); }

#define UNET_HIP(call)                                                        \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) return rtm::set_error(RTM_EHIP, hipGetErrorString(e_)); \
    } while (0)

bool ch_ok(int c) { return c == 16 || c == 32 || c == 64 || c == 128; }

bool thin_pair(int ci, int co) { return (ci == 1 && co == kThin) || (ci == kThin && co == 1); }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

int check_desc(const unet_conv_desc_t *d)
{
    if (!d) return bad("desc is NULL");
    if (d->n < 1 || d->d < 1 || d->h < 1 || d->w < 1) return bad("extents must be >= 1");
    if (!(ch_ok(d->cin) && ch_ok(d->cout)) && !thin_pair(d->cin, d->cout))
        return bad("channel counts must be 16, 32, 64 or 128, or the pair must be (1, 16) or (16, 1)");
    const int64_t nvox = (int64_t)d->n * d->d * d->h * d->w;
    if (nvox * (int64_t)(d->cin > d->cout ? d->cin : d->cout) >= ((int64_t)1 << 40))
        return bad("tensor too large");
    return RTM_OK;
}

dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

// LDS-staged forward convolution for the layers it covers (1: on), and the
// workgroup counts that choose it: a grid of one workgroup per CU already
// beats the direct kernel (measured on the 64^3 level).
std::atomic<int> g_conv_lds{1};
constexpr int64_t kLdsBlocks = 1024, kLdsMinBlocks = 256;

// Grids of fewer wavefronts than the chip has SIMDs (the coarse levels)
// split the output channels: four ways below a quarter of the SIMDs, two
// ways above (each split re-reads the activations once more).
constexpr int64_t kFwdSplitWaves = 1024;

// K split of the direct kernel on the two coarse tiers (below a quarter of
// kFwdSplitWaves wavefronts, and below kFwdSplitWaves).  Measured on the
// network's levels: four parts take the 16^3 level's forward and input
// gradient from 0.038 and 0.058 ms to 0.015 and 0.019; the 32^3 level, with
// twice as many wavefronts per CU already, gains nothing from two parts
// and loses up to 40% with four.
constexpr int kKsQuarter = 4, kKsHalf = 1;

template <int CI, int CO, int CBW, int KS>
void launch_direct(ConvArgs a, int64_t waves, hipStream_t st)
{
    const int64_t blocks = (waves * KS + 3) / 4;
    a.nblocks = (blocks + kNumXcd - 1) / kNumXcd * kNumXcd;
    hipLaunchKernelGGL((conv_fwd_kernel<CI, CO, CBW, KS>), dim3((unsigned)a.nblocks, CO / 16 / CBW), dim3(256), 0, st,
                       a);
}

template <int CI, int CO>
void launch_fwd_t(const ConvArgs &a, hipStream_t st)
{
    constexpr int CB = CO / 16, CBW4 = CB >= 4 ? CB / 4 : 1, CBW2 = CB >= 2 ? CB / 2 : 1;
    // Pairs of <= 32 channels, and 64 -> 32: its three-plane ring takes 152
    // KB of LDS (one workgroup per CU) and still halves the direct kernel's
    // time, whose 64-channel operand fragments are re-read for every tap.
    if constexpr ((CI <= 32 && CO <= 32) || (CI == 64 && CO == 32)) {
        // z-chunks sized for about kLdsBlocks workgroups, 4 to 16 planes;
        // grids that give fewer than kLdsMinBlocks take the direct kernel
        const int tx = (a.w + kLdsX - 1) / kLdsX, ty = (a.h + kLdsY - 1) / kLdsY;
        const int64_t nsamp = a.nvox / ((int64_t)a.d * a.h * a.w);
        const int64_t cols = (int64_t)tx * ty * nsamp;
        const int lz = (int)std::min<int64_t>(16, std::max<int64_t>(4, cols * a.d / kLdsBlocks));
        const int tz = (a.d + lz - 1) / lz;
        const int64_t tiles = cols * tz;
        if (a.w >= kLdsX && tiles >= kLdsMinBlocks && g_conv_lds.load()) {
            ConvArgs b = a;
            b.nblocks = (tiles + kNumXcd - 1) / kNumXcd * kNumXcd;
            hipLaunchKernelGGL((conv_fwd_lds_kernel<CI, CO>), dim3((unsigned)b.nblocks), dim3(256), 0, st, b, tx, ty,
                               tz, lz, tiles);
            return;
        }
    }
    const int64_t waves = (a.nvox + 63) / 64;
    if (CB > 1 && waves < kFwdSplitWaves / 4)
        launch_direct<CI, CO, CBW4, kKsQuarter>(a, waves, st);
    else if (CB > 1 && waves < kFwdSplitWaves)
        launch_direct<CI, CO, CBW2, kKsHalf>(a, waves, st);
    else
        launch_direct<CI, CO, CB, 1>(a, waves, st);
}

template <int CI>
int launch_fwd_ci(int co, const ConvArgs &a, hipStream_t st)
{
    switch (co) {
    case 16: launch_fwd_t<CI, 16>(a, st); return 0;
    case 32: launch_fwd_t<CI, 32>(a, st); return 0;
    case 64: launch_fwd_t<CI, 64>(a, st); return 0;
    case 128: launch_fwd_t<CI, 128>(a, st); return 0;
    }
    return -1;
}

int launch_fwd(int ci, int co, ConvArgs a, hipStream_t st)
{
    if (ci == 1 && co == kThin) {
        hipLaunchKernelGGL(conv_thin_in_kernel, grid1(a.nvox), dim3(256), 0, st, a);
        return 0;
    }
    if (ci == kThin && co == 1) {
        hipLaunchKernelGGL(conv_thin_out_kernel, grid1(a.nvox), dim3(256), 0, st, a);
        return 0;
    }
    const int64_t waves = (a.nvox + 63) / 64;
    const int64_t blocks = (waves + 3) / 4;
    a.nblocks = (blocks + kNumXcd - 1) / kNumXcd * kNumXcd;
    switch (ci) {
    case 16: return launch_fwd_ci<16>(co, a, st);
    case 32: return launch_fwd_ci<32>(co, a, st);
    case 64: return launch_fwd_ci<64>(co, a, st);
    case 128: return launch_fwd_ci<128>(co, a, st);
    }
    return -1;
}

// Row splits of the weight gradient: enough workgroups to fill the chip
// (9 x splits) while every group keeps >= 8 rows (16 with 128 input
// channels) and the partial sums stay within a fixed budget.  Each split
// writes a whole partial weight gradient, so on the coarse grids, where a
// split covers a few hundred voxels, the partials are most of the traffic:
// measured on the 16^3 and 32^3 levels, 8 and 16 rows beat 4 (and 16 rows
// lose at 32 channels).
constexpr int kWgMaxSplits = 512;
constexpr int64_t kWgPartBudget = (int64_t)64 << 20;

template <int CI, int CO>
int wg_splits(int64_t rows)
{
    constexpr int RS = WgCfg<CI, CO>::RS;
    int64_t s = rows / ((CI >= 128 ? 16 : 8) * RS);
    const int64_t by_budget = kWgPartBudget / ((int64_t)RS * 27 * CI * CO * (int64_t)sizeof(float));
    if (s > by_budget) s = by_budget;
    if (s > kWgMaxSplits) s = kWgMaxSplits;
    if (s < 1) s = 1;
    return (int)s;
}

template <int CI, int CO>
void wg_sizes(int64_t rows, int64_t *parts, int *S)
{
    *S = wg_splits<CI, CO>(rows);
    *parts = (int64_t)*S * WgCfg<CI, CO>::RS;
}

template <int CI>
int wg_sizes_ci(int co, int64_t rows, int64_t *parts, int *S)
{
    switch (co) {
    case 16: wg_sizes<CI, 16>(rows, parts, S); return 0;
    case 32: wg_sizes<CI, 32>(rows, parts, S); return 0;
    case 64: wg_sizes<CI, 64>(rows, parts, S); return 0;
    case 128: wg_sizes<CI, 128>(rows, parts, S); return 0;
    }
    return -1;
}

// One-channel layers on the matrix cores: jobs as in the ring kernel (4
// planes, 32-voxel x segments, y ranges of >= kThinMinRows rows), about
// kThinMfmaBlocks of them; one partial per wavefront (4 per job).
constexpr int64_t kThinMfmaBlocks = 2048;
constexpr int kThinMinRows = 8;

void thin_layout(const unet_conv_desc_t *d, int *nzb, int *nxs, int *ys)
{
    *nzb = (d->d + kThinZB - 1) / kThinZB;
    *nxs = (d->w + kThinSeg - 1) / kThinSeg;
    const int64_t cols = (int64_t)d->n * *nzb * *nxs;
    int64_t y = (kThinMfmaBlocks + cols - 1) / cols;
    if (y > d->h / kThinMinRows) y = d->h / kThinMinRows;
    *ys = (int)(y < 1 ? 1 : y);
}

// Ring-staged weight gradient: MFMA pairs of <= 64 input channels on grids
// of at least kRingMinVox voxels (the 64^3 and 128^3 levels of the
// network).  Jobs: (n, z block, x segment, y range), enough of them for
// about ring_blocks(cin) blocks with every y range >= kRingMinRows rows, and
// the partial sums within the weight-gradient budget.  Measured: 16 input
// channels (four-plane blocks of little work) want 512 blocks, 32 and 64
// want 256 (fewer partials; 384 or 128 blocks split the y extent unevenly and
// lose 30-90%).
constexpr int64_t kRingMinVox = (int64_t)1 << 17;
int64_t ring_blocks(int cin) { return cin == 16 ? 512 : 256; }
constexpr int kRingMinRows = 8;

// Output planes per job: four for every channel count (measured at 128^3
// and 64^3: two planes cost c7 +24%; four instead of two for 64 input
// channels, with its 96 KB ring and one workgroup per CU, cut c6 by 9%;
// eight gain c7 1% and cost c2 24%).
int ring_zb(int) { return 4; }

// Job counts of the ring kernel, or false when it does not apply.
bool ring_layout(const unet_conv_desc_t *d, int *nzb, int *nxs, int *ys)
{
    if (thin_pair(d->cin, d->cout) || d->cin > 64 || (int64_t)d->n * d->d * d->h * d->w < kRingMinVox) return false;
    *nzb = (d->d + ring_zb(d->cin) - 1) / ring_zb(d->cin);
    *nxs = (d->w + 31) / 32;
    const int64_t cols = (int64_t)d->n * *nzb * *nxs, cbs = d->cout / 16;
    const int64_t per_part = (int64_t)27 * d->cin * d->cout * (int64_t)sizeof(float);
    if (cols * per_part > kWgPartBudget) return false;
    int64_t y = (ring_blocks(d->cin) + cols * cbs - 1) / (cols * cbs);
    if (y > d->h / kRingMinRows) y = d->h / kRingMinRows;
    if (y > kWgPartBudget / (cols * per_part)) y = kWgPartBudget / (cols * per_part);
    *ys = (int)(y < 1 ? 1 : y);
    return true;
}

int wg_layout(const unet_conv_desc_t *d, int64_t *parts, int *S)
{
    const int64_t rows = (int64_t)d->n * d->d * d->h;
    int nzb, nxs, ys;
    if (ring_layout(d, &nzb, &nxs, &ys)) {
        *S = (int)((int64_t)d->n * nzb * nxs * ys);
        *parts = *S;
        return 0;
    }
    if (thin_pair(d->cin, d->cout)) {
        thin_layout(d, &nzb, &nxs, &ys);
        *S = (int)((int64_t)d->n * nzb * nxs * ys);
        *parts = (int64_t)*S * kThinZB;
        return 0;
    }
    switch (d->cin) {
    case 16: return wg_sizes_ci<16>(d->cout, rows, parts, S);
    case 32: return wg_sizes_ci<32>(d->cout, rows, parts, S);
    case 64: return wg_sizes_ci<64>(d->cout, rows, parts, S);
    case 128: return wg_sizes_ci<128>(d->cout, rows, parts, S);
    }
    return -1;
}

size_t rnd256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace: weight partials [parts][Cout*27*Cin], bias partials
// [parts][Cout], then the chunk sums of the two-pass reduction.
size_t wg_bytes(const unet_conv_desc_t *d, int64_t parts)
{
    const size_t nw = (size_t)d->cout * 27 * d->cin;
    const size_t q = (size_t)((parts + sum_chunk(parts) - 1) / sum_chunk(parts));
    return rnd256(parts * nw * sizeof(float)) + rnd256(parts * d->cout * sizeof(float)) +
           rnd256(q * nw * sizeof(float)) + rnd256(q * d->cout * sizeof(float));
}

template <int CI, int CO>
void launch_wg_t(const WgArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((conv_wgrad_kernel<CI, CO>), dim3((unsigned)a.S, 9), dim3(256), 0, st, a);
}

template <int CI>
int launch_wg_ci(int co, const WgArgs &a, hipStream_t st)
{
    switch (co) {
    case 16: launch_wg_t<CI, 16>(a, st); return 0;
    case 32: launch_wg_t<CI, 32>(a, st); return 0;
    case 64: launch_wg_t<CI, 64>(a, st); return 0;
    case 128: launch_wg_t<CI, 128>(a, st); return 0;
    }
    return -1;
}

int launch_wg(int ci, int co, const WgArgs &a, hipStream_t st)
{
    switch (ci) {
    case 16: return launch_wg_ci<16>(co, a, st);
    case 32: return launch_wg_ci<32>(co, a, st);
    case 64: return launch_wg_ci<64>(co, a, st);
    case 128: return launch_wg_ci<128>(co, a, st);
    }
    return -1;
}

int check_resample(int n, int d, int h, int w, int c)
{
    if (n < 1 || d < 1 || h < 1 || w < 1) return bad("extents must be >= 1");
    if (c < 8 || c % 8) return bad("channels must be a positive multiple of 8");
    return RTM_OK;
}

// The parts of a weight-gradient workspace (layout at wg_bytes).
struct WgWs {
    float *part, *bpart, *tmp_w, *tmp_b;
    int64_t parts, nw;
    int S;
};

int wg_ws_split(const unet_conv_desc_t *desc, void *ws, size_t ws_bytes, WgWs *o)
{
    if (wg_layout(desc, &o->parts, &o->S)) return bad("unsupported channel pair");
    if (!ws || ws_bytes < wg_bytes(desc, o->parts) || ((uintptr_t)ws & 255u))
        return rtm::set_error(RTM_EWORKSPACE, "workspace missing, too small or not 256-byte aligned");
    o->nw = (int64_t)desc->cout * 27 * desc->cin;
    const int64_t q = (o->parts + sum_chunk(o->parts) - 1) / sum_chunk(o->parts);
    char *base = static_cast<char *>(ws);
    o->part = reinterpret_cast<float *>(base);
    base += rnd256(o->parts * o->nw * sizeof(float));
    o->bpart = reinterpret_cast<float *>(base);
    base += rnd256(o->parts * desc->cout * sizeof(float));
    o->tmp_w = reinterpret_cast<float *>(base);
    base += rnd256(q * o->nw * sizeof(float));
    o->tmp_b = reinterpret_cast<float *>(base);
    return RTM_OK;
}

// The split-K pass: one partial weight and bias gradient per part.
void wg_partials(const unet_conv_desc_t *desc, const uint16_t *x, const uint16_t *dy, const WgWs &w, hipStream_t st)
{
    WgArgs a{};
    a.x = x;
    a.dy = dy;
    a.part = w.part;
    a.bpart = w.bpart;
    a.rows = (int64_t)desc->n * desc->d * desc->h;
    a.d = desc->d;
    a.h = desc->h;
    a.w = desc->w;
    a.S = w.S;
    int nzb, nxs, ys;
    if (ring_layout(desc, &nzb, &nxs, &ys)) {
        WrArgs r{};
        r.x = x;
        r.dy = dy;
        r.part = a.part;
        r.bpart = a.bpart;
        r.d = desc->d;
        r.h = desc->h;
        r.w = desc->w;
        r.cout = desc->cout;
        r.nzb = nzb;
        r.nxs = nxs;
        r.ys = ys;
        const dim3 grid((unsigned)w.S, (unsigned)(desc->cout / 16));
        switch (desc->cin) {
        case 16: hipLaunchKernelGGL((conv_wgrad_ring_kernel<16, 4>), grid, dim3(576), 0, st, r); break;
        case 32: hipLaunchKernelGGL((conv_wgrad_ring_kernel<32, 4>), grid, dim3(576), 0, st, r); break;
        default: hipLaunchKernelGGL((conv_wgrad_ring_kernel<64, 4>), grid, dim3(576), 0, st, r); break;
        }
    } else if (thin_pair(desc->cin, desc->cout)) {
        WtArgs t{};
        const bool in1 = desc->cin == 1;
        t.w16 = in1 ? dy : x;
        t.t1 = in1 ? x : dy;
        t.part = a.part;
        t.bpart = a.bpart;
        t.d = desc->d;
        t.h = desc->h;
        t.w = desc->w;
        thin_layout(desc, &t.nzb, &t.nxs, &t.ys);
        if (in1)
            hipLaunchKernelGGL(wgrad_thin_mfma_kernel<true>, dim3((unsigned)w.S), dim3(256), 0, st, t);
        else
            hipLaunchKernelGGL(wgrad_thin_mfma_kernel<false>, dim3((unsigned)w.S), dim3(256), 0, st, t);
    } else
        launch_wg(desc->cin, desc->cout, a, st);
}

int wg_check(const unet_conv_desc_t *desc, const uint16_t *x, const uint16_t *dy)
{
    if (int e = check_desc(desc)) return e;
    if (!x || !dy) return bad("x and dy are required");
    if (!aligned16(x) || !aligned16(dy)) return bad("x and dy must be 16-byte aligned");
    return RTM_OK;
}

}  // namespace

extern "C" {

int unet_weight_pack(const unet_conv_desc_t *desc, const float *w, uint16_t *w_fwd, uint16_t *w_bwd, void *stream)
{
    rtm::clear_error();
    if (int e = check_desc(desc)) return e;
    if (!w) return bad("w is NULL");
    const int64_t n = (int64_t)desc->cout * 27 * desc->cin;
    hipLaunchKernelGGL(weight_pack_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, w, desc->cin, desc->cout,
                       w_fwd, w_bwd);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_weight_pack_many(int32_t count, const unet_pack_item_t *items, void *stream)
{
    rtm::clear_error();
    if (count < 1 || count > UNET_PACK_MAX || !items) return bad("count must be in [1, UNET_PACK_MAX], items non-NULL");
    PackSet P{};
    P.count = count;
    P.start[0] = 0;
    for (int k = 0; k < count; ++k) {
        const unet_pack_item_t &L = items[k];
        if (!L.w || L.cin < 1 || L.cout < 1) return bad("each item needs w and positive channel counts");
        P.item[k] = L;
        P.start[k + 1] = P.start[k] + (int64_t)L.cout * 27 * L.cin;
    }
    bool small = true;
    for (int k = 0; k < count; ++k) small = small && P.start[k + 1] - P.start[k] < ((int64_t)1 << 32);
    if (small)
        hipLaunchKernelGGL(weight_pack_many_kernel<true>, grid1(P.start[count]), dim3(256), 0, (hipStream_t)stream, P);
    else
        hipLaunchKernelGGL(weight_pack_many_kernel<false>, grid1(P.start[count]), dim3(256), 0, (hipStream_t)stream, P);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_conv3d_fwd(const unet_conv_desc_t *desc, const uint16_t *x, const uint16_t *w_fwd, const float *bias,
                    int32_t relu, const uint16_t *skip, float *y, int32_t y_channels, uint16_t *r, uint16_t *out,
                    void *stream)
{
    rtm::clear_error();
    if (int e = check_desc(desc)) return e;
    if (!x || !w_fwd) return bad("x and w_fwd are required");
    if (!y && !r && !out) return bad("no output requested");
    if (y && (y_channels < 1 || y_channels > desc->cout)) return bad("y_channels must be in [1, cout]");
    if (skip && !out) return bad("skip needs out");
    if (!aligned16(x) || !aligned16(w_fwd)) return bad("x and w_fwd must be 16-byte aligned");
    if (desc->cin == 1 && !(aligned16(y) && aligned16(r) && aligned16(out) && aligned16(skip)))
        return bad("for the (1, 16) pair y, r, out and skip must be 16-byte aligned");
    ConvArgs a{};
    a.x = x;
    a.wt = w_fwd;
    a.bias = bias;
    a.skip = skip;
    a.y = y;
    a.r = r;
    a.out = out;
    a.nvox = (int64_t)desc->n * desc->d * desc->h * desc->w;
    a.d = desc->d;
    a.h = desc->h;
    a.w = desc->w;
    a.relu = relu ? 1 : 0;
    a.ych = y ? y_channels : 0;
    if (launch_fwd(desc->cin, desc->cout, a, (hipStream_t)stream)) return bad("unsupported channel pair");
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_set_conv_lds(int32_t lds)
{
    rtm::clear_error();
    if (lds != 0 && lds != 1) return bad("lds must be 0 or 1");
    g_conv_lds = lds;
    return RTM_OK;
}

int unet_get_conv_lds(int32_t *lds)
{
    rtm::clear_error();
    if (!lds) return bad("NULL output");
    *lds = g_conv_lds.load();
    return RTM_OK;
}

static int dgrad_impl(const unet_conv_desc_t *desc, const uint16_t *dy, const uint16_t *w_bwd, float *dx,
                      const uint16_t *mask, uint16_t *g_out, void *stream)
{
    rtm::clear_error();
    if (int e = check_desc(desc)) return e;
    if (!dy || !w_bwd || !dx) return bad("dy, w_bwd and dx are required");
    if (!aligned16(dy) || !aligned16(w_bwd)) return bad("dy and w_bwd must be 16-byte aligned");
    if (desc->cout == 1 && !aligned16(dx)) return bad("for the (16, 1) pair dx must be 16-byte aligned");
    if ((mask != nullptr) != (g_out != nullptr)) return bad("mask and g_out go together");
    if (mask && (!aligned16(mask) || !aligned16(g_out) || desc->cin % 8 != 0))
        return bad("mask and g_out must be 16-byte aligned, with a multiple of 8 input channels");
    ConvArgs a{};
    a.x = dy;
    a.wt = w_bwd;
    a.y = dx;
    a.mask = mask;
    a.gout = g_out;
    a.nvox = (int64_t)desc->n * desc->d * desc->h * desc->w;
    a.d = desc->d;
    a.h = desc->h;
    a.w = desc->w;
    a.ych = desc->cin;
    if (launch_fwd(desc->cout, desc->cin, a, (hipStream_t)stream)) return bad("unsupported channel pair");
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_conv3d_dgrad(const unet_conv_desc_t *desc, const uint16_t *dy, const uint16_t *w_bwd, float *dx,
                      void *stream)
{
    return dgrad_impl(desc, dy, w_bwd, dx, nullptr, nullptr, stream);
}

int unet_conv3d_dgrad_relu(const unet_conv_desc_t *desc, const uint16_t *dy, const uint16_t *w_bwd, float *dx,
                           const uint16_t *mask, uint16_t *g_out, void *stream)
{
    if (!mask || !g_out) {
        rtm::clear_error();
        return bad("mask and g_out are required");
    }
    return dgrad_impl(desc, dy, w_bwd, dx, mask, g_out, stream);
}

int unet_wgrad_ws_bytes(const unet_conv_desc_t *desc, size_t *bytes)
{
    rtm::clear_error();
    if (int e = check_desc(desc)) return e;
    if (!bytes) return bad("bytes is NULL");
    int64_t parts;
    int S;
    if (wg_layout(desc, &parts, &S)) return bad("unsupported channel pair");
    *bytes = wg_bytes(desc, parts);
    return RTM_OK;
}


int unet_conv3d_wgrad(const unet_conv_desc_t *desc, const uint16_t *x, const uint16_t *dy, float *dw, float *db,
                      void *ws, size_t ws_bytes, void *stream)
{
    rtm::clear_error();
    if (int e = wg_check(desc, x, dy)) return e;
    if (!dw) return bad("dw is required");
    WgWs w;
    if (int e = wg_ws_split(desc, ws, ws_bytes, &w)) return e;
    hipStream_t st = (hipStream_t)stream;
    wg_partials(desc, x, dy, w, st);
    UNET_HIP(sum_parts(w.part, w.nw, w.tmp_w, dw, w.bpart, db ? desc->cout : 0, w.tmp_b, db, w.parts, st));
    return RTM_OK;
}

int unet_conv3d_wgrad_partial(const unet_conv_desc_t *desc, const uint16_t *x, const uint16_t *dy, void *ws,
                              size_t ws_bytes, void *stream)
{
    rtm::clear_error();
    if (int e = wg_check(desc, x, dy)) return e;
    WgWs w;
    if (int e = wg_ws_split(desc, ws, ws_bytes, &w)) return e;
    wg_partials(desc, x, dy, w, (hipStream_t)stream);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_wgrad_reduce_many(int32_t count, const unet_wgrad_item_t *items, void *stream)
{
    rtm::clear_error();
    if (count < 1 || count > UNET_WGRAD_MAX || !items)
        return bad("count must be in [1, UNET_WGRAD_MAX], items non-NULL");
    SumMany m1{}, m2{};
    m1.count = m2.count = count;
    for (int k = 0; k < count; ++k) {
        const unet_wgrad_item_t &it = items[k];
        if (int e = check_desc(&it.desc)) return e;
        if (!it.dw) return bad("dw is required for every item");
        WgWs w;
        if (int e = wg_ws_split(&it.desc, it.ws, it.ws_bytes, &w)) return e;
        const int64_t n1 = it.db ? it.desc.cout : 0;
        const int64_t q = (w.parts + sum_chunk(w.parts) - 1) / sum_chunk(w.parts);
        const int32_t bx = (int32_t)((w.nw + n1 + 255) / 256);
        // the two passes of sum_parts: chunks of sum_chunk(P) partials, then
        // the chunk sums
        m1.w[k] = SumSet{w.part, w.tmp_w, w.nw};
        m1.b[k] = SumSet{w.bpart, w.tmp_b, n1};
        m1.P[k] = w.parts;
        m1.chunk[k] = (int32_t)sum_chunk(w.parts);
        m1.bx[k] = bx;
        m1.start[k + 1] = m1.start[k] + (int64_t)bx * q;
        m2.w[k] = SumSet{w.tmp_w, it.dw, w.nw};
        m2.b[k] = SumSet{w.tmp_b, it.db, n1};
        m2.P[k] = q;
        m2.chunk[k] = (int32_t)q;
        m2.bx[k] = bx;
        m2.start[k + 1] = m2.start[k] + bx;
    }
    if (m1.start[count] > 0x7fffffff) return bad("reduction too large for one launch");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(sum_parts_many_kernel, dim3((unsigned)m1.start[count]), dim3(256), 0, st, m1);
    hipLaunchKernelGGL(sum_parts_many_kernel, dim3((unsigned)m2.start[count]), dim3(256), 0, st, m2);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_embed(int64_t nvox, int32_t channels, const float *img, float scale, uint16_t *x, void *stream)
{
    rtm::clear_error();
    if (nvox < 1 || channels < 1 || !img || !x) return bad("invalid embed arguments");
    if ((nvox * channels) % 8 == 0 && aligned16(x))
        hipLaunchKernelGGL(embed8_kernel, grid1(nvox * channels / 8), dim3(256), 0, (hipStream_t)stream, nvox, channels,
                           img, scale, x);
    else
        hipLaunchKernelGGL(embed_kernel, grid1(nvox * channels), dim3(256), 0, (hipStream_t)stream, nvox, channels, img,
                           scale, x);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_pool2(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const uint16_t *x, uint16_t *y, void *stream)
{
    rtm::clear_error();
    if (int e = check_resample(n, d, h, w, c)) return e;
    if ((d | h | w) & 1) return bad("pooled extents must be even");
    if (!x || !y || !aligned16(x) || !aligned16(y)) return bad("x and y must be 16-byte aligned device pointers");
    const int64_t total = (int64_t)n * (d / 2) * (h / 2) * (w / 2) * (c / 8);
    hipLaunchKernelGGL(pool2_kernel, grid1(total), dim3(256), 0, (hipStream_t)stream, n, d, h, w, c, x, y);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_up2(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const uint16_t *x, uint16_t *y, void *stream)
{
    rtm::clear_error();
    if (int e = check_resample(n, d, h, w, c)) return e;
    if (!x || !y || !aligned16(x) || !aligned16(y)) return bad("x and y must be 16-byte aligned device pointers");
    const int64_t total = (int64_t)n * 8 * d * h * w * (c / 8);
    hipLaunchKernelGGL(up2_kernel, grid1(total), dim3(256), 0, (hipStream_t)stream, n, d, h, w, c, x, y);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

static int up2_bwd_impl(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const float *g_fine, float *g_coarse,
                        const uint16_t *mask, uint16_t *g_out, void *stream)
{
    rtm::clear_error();
    if (n < 1 || d < 1 || h < 1 || w < 1 || c < 1 || !g_fine || !g_coarse) return bad("invalid up2_bwd arguments");
    const int64_t total = (int64_t)n * d * h * w * c;
    if (c % 4 == 0 && aligned8(mask) && aligned8(g_out))
        hipLaunchKernelGGL(up2_bwd_kernel<4>, grid1(total / 4), dim3(256), 0, (hipStream_t)stream, n, d, h, w, c,
                           g_fine, g_coarse, mask, g_out);
    else
        hipLaunchKernelGGL(up2_bwd_kernel<1>, grid1(total), dim3(256), 0, (hipStream_t)stream, n, d, h, w, c, g_fine,
                           g_coarse, mask, g_out);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_up2_bwd(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const float *g_fine, float *g_coarse,
                 void *stream)
{
    return up2_bwd_impl(n, d, h, w, c, g_fine, g_coarse, nullptr, nullptr, stream);
}

int unet_up2_bwd_relu(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const float *g_fine, float *g_coarse,
                      const uint16_t *mask, uint16_t *g_out, void *stream)
{
    if (!mask || !g_out) {
        rtm::clear_error();
        return bad("mask and g_out are required");
    }
    return up2_bwd_impl(n, d, h, w, c, g_fine, g_coarse, mask, g_out, stream);
}

int unet_relu_grad(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, const float *g1, const float *g2,
                   const float *g_pool, const uint16_t *mask, uint16_t *out, void *stream)
{
    rtm::clear_error();
    if (n < 1 || d < 1 || h < 1 || w < 1 || c < 1 || !g1 || !mask || !out) return bad("invalid relu_grad arguments");
    if (g_pool && ((d | h | w) & 1)) return bad("g_pool needs even extents");
    const int64_t total = (int64_t)n * d * h * w * c;
    if (c % 4 == 0 && aligned8(mask) && aligned8(out))
        hipLaunchKernelGGL(relu_grad_kernel<4>, grid1(total / 4), dim3(256), 0, (hipStream_t)stream, n, d, h, w, c, g1,
                           g2, g_pool, mask, out);
    else
        hipLaunchKernelGGL(relu_grad_kernel<1>, grid1(total), dim3(256), 0, (hipStream_t)stream, n, d, h, w, c, g1, g2,
                           g_pool, mask, out);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_mse_ws_bytes(int64_t nvox, size_t *bytes)
{
    rtm::clear_error();
    if (nvox < 1 || !bytes) return bad("invalid mse_ws_bytes arguments");
    *bytes = (kMseBlocks + 1) * sizeof(double);
    return RTM_OK;
}

int unet_mse(int64_t nvox, int32_t channels, const float *img, const float *y, const float *target, float *out,
             uint16_t *gy, double *loss, void *ws, size_t ws_bytes, void *stream)
{
    rtm::clear_error();
    if (nvox < 1 || channels < 1 || !img || !y) return bad("invalid mse arguments");
    if ((gy || loss) && !target) return bad("gy and loss need target");
    if (target && (!ws || ws_bytes < (kMseBlocks + 1) * sizeof(double)))
        return rtm::set_error(RTM_EWORKSPACE, "workspace missing or too small");
    hipStream_t st = (hipStream_t)stream;
    double *part = static_cast<double *>(ws);
    int nb;
    if (channels == 1 && nvox % 4 == 0 && aligned16(img) && aligned16(y) && aligned16(target) && aligned16(out) &&
        aligned8(gy)) {
        nb = (int)std::min<int64_t>(kMseBlocks, (nvox / 4 + 255) / 256);
        hipLaunchKernelGGL(mse4_kernel, dim3(nb), dim3(256), 0, st, nvox, img, y, target, out, gy, part);
    } else {
        nb = (int)std::min<int64_t>(kMseBlocks, (nvox + 255) / 256);
        hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, st, nvox, channels, img, y, target, out, gy, part);
    }
    if (target) {
        hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, part, nb, nvox, part + kMseBlocks);
        if (loss) {
            UNET_HIP(hipMemcpyAsync(loss, part + kMseBlocks, sizeof(double), hipMemcpyDeviceToHost, st));
            UNET_HIP(hipStreamSynchronize(st));
        }
    }
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

int unet_adam(int64_t n, float *p, const float *g, float *m, float *v, double lr, double b1, double b2, double eps,
              int32_t step, void *stream)
{
    rtm::clear_error();
    if (n < 1 || !p || !g || !m || !v) return bad("invalid adam arguments");
    if (step < 1 || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) || !(eps > 0.0))
        return bad("adam needs step >= 1, 0 <= b1, b2 < 1, eps > 0");
    // 1 - b and the bias corrections are formed in double: 1 - b in float32
    // from a float32 b (0.999 -> 0.99900001) loses 4 digits.
    const float c1 = (float)(1.0 - std::pow(b1, step));
    const float c2 = (float)(1.0 - std::pow(b2, step));
    const float omb1 = (float)(1.0 - b1), omb2 = (float)(1.0 - b2);
    hipLaunchKernelGGL(adam_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, n, p, g, m, v, (float)lr, (float)b1,
                       (float)b2, omb1, omb2, (float)eps, c1, c2);
    UNET_HIP(hipGetLastError());
    return RTM_OK;
}

}  // extern "C"

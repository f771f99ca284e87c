// Auxiliary kernels of librtm: random boundary padding and its adjoint,
// preparation of the scaled velocity term, trace transposes, receiver-field
// start, last-sample recording, image and gradient finalisation, and field
// unpacking.  All run once per call (not per time step).
#include <algorithm>

#include "common.h"

namespace rtm {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t gid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

inline unsigned grid_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (unsigned)b;
}

// Grid for reductions: a few blocks per CU, each striding over the data.
inline unsigned grid_reduce(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (unsigned)b;
}

// SplitMix64 (Steele, Lea & Flood 2014): output number k + 1 of the stream
// seeded with `seed` (state advanced by the golden-ratio increment, then the
// 64-bit finaliser).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Random factor of band cell j, uniform in [0.7, 1.3): one FP32 fma of the
// exact 24-bit fraction.
__device__ __forceinline__ float rbc_factor(uint64_t seed, uint64_t j)
{
    const float u = (float)(splitmix64_at(seed, j) >> 40) * (1.0f / 16777216.0f);
    return __builtin_fmaf(0.6f, u, 0.7f);
}

struct PadDims {
    int ndim;
    int nb;
    int64_t nx, ny, nz;
    int64_t NX, NY, NZ;
};

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Distance of a padded coordinate from the interior [0, n) along one axis.
__device__ __forceinline__ int64_t band_depth(int64_t a, int64_t n) { return a < 0 ? -a : (a >= n ? a - n + 1 : 0); }

// Depth of a band cell: the largest per-axis distance from the interior.
__device__ __forceinline__ int64_t cell_depth(const PadDims &d, int64_t ix, int64_t iy, int64_t iz)
{
    int64_t m = band_depth(ix, d.nx);
    m = max(m, band_depth(iz, d.nz));
    if (d.ndim == 3) m = max(m, band_depth(iy, d.ny));
    return m;
}

// Block-wide max / min of unsigned values (kBlock threads), then one
// atomic per block.
template <bool MAX>
__device__ __forceinline__ void block_reduce_atomic(unsigned m, unsigned *out)
{
    __shared__ unsigned part[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        unsigned o = (unsigned)__shfl_xor((int)m, off);
        m = MAX ? max(m, o) : min(m, o);
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = MAX ? max(m, part[w]) : min(m, part[w]);
        if (MAX) atomicMax(out, m);
        else atomicMin(out, m);
    }
}

__global__ __launch_bounds__(kBlock) void vmax_bits_kernel(const float *__restrict__ v, int64_t n,
                                                           unsigned *__restrict__ out)
{
    // Largest IEEE bit pattern: for positive finite data it is the maximum;
    // a NaN, infinity or negative value compares above +inf's pattern.
    unsigned m = 0u;
    for (int64_t i = gid(); i < n; i += gstride()) m = max(m, __float_as_uint(v[i]));
    block_reduce_atomic<true>(m, out);
}

__global__ __launch_bounds__(kBlock) void vmin_bits_kernel(const float *__restrict__ v, int64_t n,
                                                           unsigned *__restrict__ out)
{
    unsigned m = 0xffffffffu;
    for (int64_t i = gid(); i < n; i += gstride()) m = min(m, __float_as_uint(v[i]));
    block_reduce_atomic<false>(m, out);
}

__global__ void set_u32_kernel(unsigned *__restrict__ p, int n, unsigned v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Band cell value: min(f_j v_edge, cap); with the taper min(c_i (f_j v_edge),
// cap) at depth i; 0 above the interior with the free surface.
__global__ void rbc_pad_kernel(PadDims d, const float *__restrict__ v_int, uint64_t seed, float v_cap,
                               const unsigned *__restrict__ cap_bits, BandOpts o, float *__restrict__ v_pad)
{
    const float cap = cap_bits ? __uint_as_float(*cap_bits) : v_cap;
    const int64_t n = d.NX * d.NY * d.NZ;
    for (int64_t j = gid(); j < n; j += gstride()) {
        const int64_t x = j % d.NX;
        const int64_t y = (j / d.NX) % d.NY;
        const int64_t z = j / (d.NX * d.NY);
        const int64_t ix = x - d.nb, iz = z - d.nb, iy = (d.ndim == 3) ? y - d.nb : 0;
        const bool inside = ix >= 0 && ix < d.nx && iy >= 0 && iy < d.ny && iz >= 0 && iz < d.nz;
        const int64_t e = (clampi(iz, 0, d.nz - 1) * d.ny + clampi(iy, 0, d.ny - 1)) * d.nx + clampi(ix, 0, d.nx - 1);
        const float ve = v_int[e];
        if (inside) {
            v_pad[j] = ve;
        } else if ((o.flags & kBandFreeSurface) && iz < 0) {
            v_pad[j] = 0.f;
        } else {
            const float f = rbc_factor(seed, (uint64_t)j);
            float v = __fmul_rn(f, ve);
            if (o.flags & kBandTaper) v = __fmul_rn(o.c[cell_depth(d, ix, iy, iz) - 1], v);
            v_pad[j] = fminf(v, cap);
        }
    }
}

// Gather form of the padding adjoint: each interior cell collects its own
// gradient and (c_i) f_j times the gradient of every uncapped band cell j
// whose clamped coordinates are this cell (free-surface cells are constant).
__global__ void pad_adjoint_kernel(PadDims d, const float *__restrict__ v_int, uint64_t seed, float v_cap,
                                   const unsigned *__restrict__ cap_bits, BandOpts o,
                                   const float *__restrict__ g_pad, float *__restrict__ g_int)
{
    const float cap = cap_bits ? __uint_as_float(*cap_bits) : v_cap;
    const int64_t n = d.nx * d.ny * d.nz;
    for (int64_t i = gid(); i < n; i += gstride()) {
        const int64_t ix = i % d.nx;
        const int64_t iy = (i / d.nx) % d.ny;
        const int64_t iz = i / (d.nx * d.ny);
        const float ve = v_int[i];
        // Padded coordinate ranges that clamp onto (iz, iy, ix).
        const int64_t xlo = (ix == 0) ? 0 : ix + d.nb, xhi = (ix == d.nx - 1) ? d.NX - 1 : ix + d.nb;
        const int64_t zlo = (iz == 0) ? 0 : iz + d.nb, zhi = (iz == d.nz - 1) ? d.NZ - 1 : iz + d.nb;
        int64_t ylo = 0, yhi = 0;
        if (d.ndim == 3) {
            ylo = (iy == 0) ? 0 : iy + d.nb;
            yhi = (iy == d.ny - 1) ? d.NY - 1 : iy + d.nb;
        }
        const int64_t cx = ix + d.nb, cz = iz + d.nb, cy = (d.ndim == 3) ? iy + d.nb : 0;
        float acc = 0.f;
        for (int64_t z = zlo; z <= zhi; ++z)
            for (int64_t y = ylo; y <= yhi; ++y)
                for (int64_t x = xlo; x <= xhi; ++x) {
                    const int64_t j = (z * d.NY + y) * d.NX + x;
                    if (z == cz && y == cy && x == cx) {
                        acc += g_pad[j];
                    } else if (!((o.flags & kBandFreeSurface) && z < d.nb)) {
                        float f = rbc_factor(seed, (uint64_t)j);
                        float v = __fmul_rn(f, ve);
                        if (o.flags & kBandTaper) {
                            const float c = o.c[cell_depth(d, x - d.nb, (d.ndim == 3) ? y - d.nb : 0, z - d.nb) - 1];
                            v = __fmul_rn(c, v);
                            f = __fmul_rn(c, f);
                        }
                        if (v < cap) acc = fmaf(f, g_pad[j], acc);
                    }
                }
        g_int[i] = acc;
    }
}

__global__ void fill_kernel(float *__restrict__ p, int64_t n, float v)
{
    for (int64_t i = gid(); i < n; i += gstride()) p[i] = v;
}

// D'[cell] = (v dt / h)^2 on the padded grid, zero in the halo.
__global__ void build_dp_kernel(Layout L, const float *__restrict__ v_pad, float dt_over_h, float *__restrict__ Dp)
{
    for (int64_t i = gid(); i < L.total; i += gstride()) {
        const int64_t zz = i / L.plane - kRadius;
        const int64_t rem = i % L.plane;
        const int64_t yy = (L.ndim == 3) ? rem / L.pitch - kRadius : 0;
        const int64_t xx = rem % L.pitch - kXOff;
        float val = 0.f;
        if (zz >= 0 && zz < L.NZ && yy >= 0 && yy < L.NY && xx >= 0 && xx < L.NX) {
            const float c = v_pad[(zz * L.NY + yy) * L.NX + xx] * dt_over_h;
            val = c * c;
        }
        Dp[i] = val;
    }
}

// Dense [NZ][NY][NX] copy of a halo-layout field.
__global__ void unpack_kernel(Layout L, const float *__restrict__ f, float *__restrict__ out)
{
    const int64_t n = (int64_t)L.NX * L.NY * L.NZ;
    for (int64_t j = gid(); j < n; j += gstride()) {
        const int64_t x = j % L.NX;
        const int64_t y = (j / L.NX) % L.NY;
        const int64_t z = j / ((int64_t)L.NX * L.NY);
        out[j] = f[L.org + z * L.plane + y * L.pitch + x];
    }
}

// out[c][r] = in[r][c] for an R x C matrix, through a 32 x 33 LDS tile.
__global__ void transpose_kernel(const float *__restrict__ in, float *__restrict__ out, int64_t R, int64_t C)
{
    __shared__ float tile[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
    for (int i = ty; i < 32; i += 8) {
        int64_t r = r0 + i, c = c0 + tx;
        if (r < R && c < C) tile[i][tx] = in[r * C + c];
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        int64_t c = c0 + i, r = r0 + tx;
        if (r < R && c < C) out[c * R + r] = tile[tx][i];
    }
}

// mu^N = D' (R^T g^N): one thread per receiver injection node, any shot.
__global__ void inj_set_kernel(const ShotDev *__restrict__ shots, const InjEnt *__restrict__ ents, int ebeg, int eend,
                               const Contrib *__restrict__ cont, int step)
{
    const int e = ebeg + (int)gid();
    if (e >= eend) return;
    const InjEnt E = ents[e];
    const ShotDev &S = shots[E.shot];
    const float *sig = S.sig + (int64_t)step * S.nrec;
    float s = 0.f;
    for (int c = E.cbeg; c < E.cend; ++c) s = fmaf(cont[c].w, sig[cont[c].idx], s);
    const int64_t off = S.L.org + (int64_t)E.z * S.L.plane + (int64_t)E.y * S.L.pitch + E.x;
    float *mu = S.fld[2 + (step & 1)];
    mu[off] = S.Dp[off] * s;
}

// d^n = R p^n for all receivers of every shot (used for the last sample).
__global__ void sample_kernel(const ShotDev *__restrict__ shots, const SampleTask *__restrict__ stasks, int n,
                              int slot)
{
    const SampleTask task = stasks[blockIdx.x];
    const ShotDev &S = shots[task.shot];
    const int r = task.r0 + (int)threadIdx.x;
    if (r >= S.nrec) return;
    const float *p = S.fld[slot] + S.L.org;
    float s = 0.f;
    for (int q = 0; q < kMaxNodes; ++q) s = fmaf(S.rw[r * kMaxNodes + q], p[S.rnode[r * kMaxNodes + q]], s);
    S.rec_out[(int64_t)n * S.nrec + r] = s;
}

// max of den over the interior box, as float bits (den >= 0).
__global__ __launch_bounds__(kBlock) void den_max_kernel(const ShotDev *__restrict__ shots, int shot, unsigned *__restrict__ out)
{
    const ShotDev &S = shots[shot];
    const int64_t nx = S.ix1 - S.ix0, ny = S.iy1 - S.iy0, nz = S.iz1 - S.iz0;
    const int64_t n = nx * ny * nz;
    unsigned m = 0u;
    for (int64_t i = gid(); i < n; i += gstride()) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        const int64_t off = S.L.org + (z + S.iz0) * S.L.plane + (y + S.iy0) * S.L.pitch + (x + S.ix0);
        m = max(m, __float_as_uint(fmaxf(S.acc1[off], 0.f)));
    }
    block_reduce_atomic<true>(m, out);
}

// image = num / (den + eps max(den)) on the interior crop (Eq. (3)).
__global__ void image_kernel(const ShotDev *__restrict__ shots, int shot, const unsigned *__restrict__ dmax_bits,
                             float eps_rel, float *__restrict__ image, int accumulate, float *__restrict__ num_out,
                             float *__restrict__ den_out)
{
    const ShotDev &S = shots[shot];
    const float stab = eps_rel * __uint_as_float(*dmax_bits);
    const int64_t nx = S.ix1 - S.ix0, ny = S.iy1 - S.iy0, nz = S.iz1 - S.iz0;
    const int64_t n = nx * ny * nz;
    for (int64_t i = gid(); i < n; i += gstride()) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        const int64_t off = S.L.org + (z + S.iz0) * S.L.plane + (y + S.iy0) * S.L.pitch + (x + S.ix0);
        const float a = S.acc0[off], b = S.acc1[off];
        if (image) {
            const float v = a / (b + stab);
            image[i] = accumulate ? image[i] + v : v;
        }
        if (num_out) num_out[i] = a;
        if (den_out) den_out[i] = b;
    }
}

// Dense interior copy of p^m (field fld[lev] of the shot table) for the
// migration with a stored source wavefield: out[(z ny + y) nx + x] = p at
// interior cell (x, y, z).
__global__ void snap_store_kernel(const ShotDev *__restrict__ shots, int shot, int lev, float *__restrict__ out)
{
    const ShotDev &S = shots[shot];
    const int64_t nx = S.ix1 - S.ix0, ny = S.iy1 - S.iy0, nz = S.iz1 - S.iz0;
    const int64_t n = nx * ny * nz;
    const float *f = S.fld[lev];
    for (int64_t i = gid(); i < n; i += gstride()) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        out[i] = f[S.L.org + (z + S.iz0) * S.L.plane + (y + S.iy0) * S.L.pitch + (x + S.ix0)];
    }
}

// flag |= 1 if any of x[0 .. n) is NaN or infinite (one atomic per block).
__global__ __launch_bounds__(kBlock) void nonfinite_kernel(const float *__restrict__ x, int64_t n,
                                                           unsigned *__restrict__ flag)
{
    unsigned m = 0u;
    for (int64_t i = gid(); i < n; i += gstride()) m = max(m, __float_as_uint(x[i]) & 0x7fffffffu);
    block_reduce_atomic<true>(m >= 0x7f800000u ? 1u : 0u, flag);
}

// grad_v = 2 G / (v^3 dt^2) on the dense padded grid.
__global__ void grad_kernel(const ShotDev *__restrict__ shots, int shot, const float *__restrict__ v_pad, float dt,
                            float *__restrict__ grad)
{
    const ShotDev &S = shots[shot];
    const Layout L = S.L;
    const int64_t n = (int64_t)L.NX * L.NY * L.NZ;
    const float two_over_dt2 = 2.0f / (dt * dt);
    for (int64_t j = gid(); j < n; j += gstride()) {
        const int64_t x = j % L.NX, y = (j / L.NX) % L.NY, z = j / ((int64_t)L.NX * L.NY);
        const float G = S.acc0[L.org + z * L.plane + y * L.pitch + x];
        const float v = v_pad[j];
        grad[j] = v > 0.f ? two_over_dt2 * G / (v * v * v) : 0.f;  // dJ/dv = 2 v dt^2 dJ/dD
    }
}

// dJ/dw^n = h^-2 sum over source nodes of the recorded coefficient * mu^{n+1}.
__global__ void wadj_kernel(const float *__restrict__ parts, int nt, float scale, float *__restrict__ out)
{
    const int n = (int)gid();
    if (n >= nt) return;
    float s = 0.f;
    for (int q = 0; q < kMaxNodes; ++q) s += parts[(int64_t)n * kMaxNodes + q];
    out[n] = s * scale;
}

// Columns [x0, x0 + w) of a [nz][nxg] array into (mode 0) or added from
// (mode 1) a dense [nz][w] window.
__global__ void window_kernel(float *__restrict__ global, const float *__restrict__ win_in,
                              float *__restrict__ win_out, int64_t nz, int64_t nxg, int64_t x0, int64_t w, int mode)
{
    const int64_t n = nz * w;
    for (int64_t i = gid(); i < n; i += gstride()) {
        const int64_t z = i / w, x = i % w;
        const int64_t g = z * nxg + x0 + x;
        if (mode == 0) win_out[i] = global[g];
        else global[g] += win_in[i];
    }
}

// Residual r = d - d_obs and per-block partial sums of r^2 (fixed order
// within a block); a second single-block pass adds the partials in order,
// so J = 0.5 sum r^2 is deterministic.
constexpr int kMisfitBlocks = 1024;

__global__ __launch_bounds__(kBlock) void misfit_partial_kernel(const float *__restrict__ d,
                                                                const float *__restrict__ dobs,
                                                                float *__restrict__ r, int64_t n,
                                                                double *__restrict__ part)
{
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int64_t i = gid(); i < n; i += gstride()) {
        const float v = d[i] - dobs[i];
        if (r) r[i] = v;
        acc += (double)v * (double)v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void misfit_final_kernel(const double *__restrict__ part, int nparts,
                                                              double *__restrict__ out)
{
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = 0.5 * sh[0];
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

static PadDims pad_dims(int ndim, int nb, int64_t nx, int64_t ny, int64_t nz)
{
    PadDims d;
    d.ndim = ndim;
    d.nb = nb;
    d.nx = nx;
    d.ny = (ndim == 3) ? ny : 1;
    d.nz = nz;
    d.NX = nx + 2 * nb;
    d.NZ = nz + 2 * nb;
    d.NY = (ndim == 3) ? ny + 2 * nb : 1;
    return d;
}

// Streaming copy of n 16-byte units: the bandwidth reference of the
// measurements (a plain read-once, write-once kernel of known size).  Each
// thread keeps kCopyUnroll independent 16-byte loads in flight; a block's
// loads of one round are contiguous (kBlock x 16 B per unrolled slot), and
// blocks stride over the buffer in whole rounds.
constexpr int kCopyUnroll = 4;
typedef float copy4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void stream_copy_kernel(const copy4 *__restrict__ src,
                                                             copy4 *__restrict__ dst, int64_t n)
{
    const int64_t round = (int64_t)kBlock * kCopyUnroll;
    for (int64_t base = (int64_t)blockIdx.x * round; base < n; base += (int64_t)gridDim.x * round) {
        copy4 v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kBlock + threadIdx.x;
            if (i < n) v[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kBlock + threadIdx.x;
            if (i < n) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
}

hipError_t launch_vrange(const float *v, int64_t n, unsigned *maxmin2, hipStream_t st)
{
    hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(64), 0, st, maxmin2, 1, 0u);
    hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(64), 0, st, maxmin2 + 1, 1, 0xffffffffu);
    hipLaunchKernelGGL(vmax_bits_kernel, dim3(grid_reduce(n)), dim3(kBlock), 0, st, v, n, maxmin2);
    hipLaunchKernelGGL(vmin_bits_kernel, dim3(grid_reduce(n)), dim3(kBlock), 0, st, v, n, maxmin2 + 1);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t units, int blocks_per_cu, hipStream_t st)
{
    if (units <= 0) return hipSuccess;
    const int64_t round = (int64_t)kBlock * kCopyUnroll;
    int64_t b = (units + round - 1) / round;
    const int64_t cap = (int64_t)256 * blocks_per_cu;
    if (b > cap) b = cap;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)b), dim3(kBlock), 0, st, (const copy4 *)src, (copy4 *)dst,
                       units);
    return hipGetLastError();
}

hipError_t launch_vmax(const float *v, int64_t n, unsigned *out, hipStream_t st)
{
    hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(64), 0, st, out, 1, 0u);
    hipLaunchKernelGGL(vmax_bits_kernel, dim3(grid_reduce(n)), dim3(kBlock), 0, st, v, n, out);
    return hipGetLastError();
}

hipError_t launch_rbc_pad(int ndim, int nb, int64_t nx, int64_t ny, int64_t nz, const float *v_int, uint64_t seed,
                          float v_cap, const unsigned *cap_bits, const BandOpts &o, float *v_pad, hipStream_t st)
{
    PadDims d = pad_dims(ndim, nb, nx, ny, nz);
    hipLaunchKernelGGL(rbc_pad_kernel, dim3(grid_for(d.NX * d.NY * d.NZ)), dim3(kBlock), 0, st, d, v_int, seed,
                       v_cap, cap_bits, o, v_pad);
    return hipGetLastError();
}

hipError_t launch_pad_adjoint(int ndim, int nb, int64_t nx, int64_t ny, int64_t nz, const float *v_int,
                              uint64_t seed, float v_cap, const unsigned *cap_bits, const BandOpts &o,
                              const float *g_pad, float *g_int, hipStream_t st)
{
    PadDims d = pad_dims(ndim, nb, nx, ny, nz);
    hipLaunchKernelGGL(pad_adjoint_kernel, dim3(grid_for(d.nx * d.ny * d.nz)), dim3(kBlock), 0, st, d, v_int, seed,
                       v_cap, cap_bits, o, g_pad, g_int);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_build_dp(const Layout &L, const float *v_pad, float dt_over_h, float *Dp, hipStream_t st)
{
    hipLaunchKernelGGL(build_dp_kernel, dim3(grid_for(L.total)), dim3(kBlock), 0, st, L, v_pad, dt_over_h, Dp);
    return hipGetLastError();
}

hipError_t launch_unpack(const Layout &L, const float *f, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(unpack_kernel, dim3(grid_for((int64_t)L.NX * L.NY * L.NZ)), dim3(kBlock), 0, st, L, f, out);
    return hipGetLastError();
}

hipError_t launch_transpose(const float *in, float *out, int64_t R, int64_t C, hipStream_t st)
{
    dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32));
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, in, out, R, C);
    return hipGetLastError();
}

hipError_t launch_inj_set(const ShotDev *shots, const InjEnt *ents, int ebeg, int eend, const Contrib *cont, int step,
                          hipStream_t st)
{
    int n = eend - ebeg;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(inj_set_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, shots, ents, ebeg, eend,
                       cont, step);
    return hipGetLastError();
}

hipError_t launch_sample(const ShotDev *shots, const SampleTask *stasks, int ntask, int n, int slot, hipStream_t st)
{
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(sample_kernel, dim3(ntask), dim3(64), 0, st, shots, stasks, n, slot);
    return hipGetLastError();
}

hipError_t launch_image(const ShotDev *shots, int shot, int64_t ninterior, unsigned *dmax_bits, float eps_rel,
                        float *image, int accumulate, float *num, float *den, hipStream_t st)
{
    hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(64), 0, st, dmax_bits, 1, 0u);
    hipLaunchKernelGGL(den_max_kernel, dim3(grid_reduce(ninterior)), dim3(kBlock), 0, st, shots, shot, dmax_bits);
    hipLaunchKernelGGL(image_kernel, dim3(grid_for(ninterior)), dim3(kBlock), 0, st, shots, shot,
                       (const unsigned *)dmax_bits, eps_rel, image, accumulate, num, den);
    return hipGetLastError();
}

hipError_t launch_snap_store(const ShotDev *shots, int shot, int lev, int64_t ninterior, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(snap_store_kernel, dim3(grid_for(ninterior)), dim3(kBlock), 0, st, shots, shot, lev, out);
    return hipGetLastError();
}

hipError_t launch_nonfinite(const float *x, int64_t n, unsigned *flag, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_reduce(n)), dim3(kBlock), 0, st, x, n, flag);
    return hipGetLastError();
}

hipError_t launch_grad(const ShotDev *shots, int shot, int64_t npad, const float *v_pad, float dt, float *grad,
                       hipStream_t st)
{
    hipLaunchKernelGGL(grad_kernel, dim3(grid_for(npad)), dim3(kBlock), 0, st, shots, shot, v_pad, dt, grad);
    return hipGetLastError();
}

hipError_t launch_window(float *global, const float *win_in, float *win_out, int64_t nz, int64_t nxg, int64_t x0,
                         int64_t w, int mode, hipStream_t st)
{
    hipLaunchKernelGGL(window_kernel, dim3(grid_for(nz * w)), dim3(kBlock), 0, st, global, win_in, win_out, nz, nxg, x0,
                       w, mode);
    return hipGetLastError();
}

size_t misfit_ws_bytes() { return sizeof(double) * (kMisfitBlocks + 1); }

hipError_t launch_misfit(const float *d, const float *dobs, float *r, int64_t n, void *ws, double *J, hipStream_t st)
{
    double *part = (double *)ws;
    const unsigned nb = std::min<int64_t>(kMisfitBlocks, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(misfit_partial_kernel, dim3(nb), dim3(kBlock), 0, st, d, dobs, r, n, part);
    hipLaunchKernelGGL(misfit_final_kernel, dim3(1), dim3(kBlock), 0, st, (const double *)part, (int)nb, J);
    return hipGetLastError();
}

hipError_t launch_wadj(const float *parts, int nt, float scale, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(wadj_kernel, dim3((nt + kBlock - 1) / kBlock), dim3(kBlock), 0, st, parts, nt, scale, out);
    return hipGetLastError();
}

}  // namespace rtm

// 2-D propagation kernels for gfx950.
//
// One wavefront (64 lanes) owns a strip of 64 * VEC consecutive x cells and
// marches down the rows [z0, z1) of its tile.  Each lane keeps the nine rows
// z-4 .. z+4 of its VEC cells in registers (a register queue), so every
// stored value of the input field is read from memory once per tile plus the
// 8-row overlap with the tiles above and below.  The x-neighbours of the
// centre row come from the adjacent lanes through DPP wave shifts; lanes 0
// and 63 supply the 4-cell halo at the strip ends from one extra load.
//
// The stencil is evaluated as a sum of differences,
//   L p_i = sum_axis sum_{m=1..4} c_m ((p_{i+m} - p_i) + (p_{i-m} - p_i)),
// which is algebraically the 8th-order Laplacian of Sec. 3 but annihilates
// constants exactly in FP32: the rounded weights then cannot add a spurious
// mass term, which would otherwise accumulate into a phase error of ~1e-3
// after a few thousand steps.
//
// Fields are stored with a zero halo and the scaled velocity term
// D' = (v dt / h)^2 is zero there, so updating a halo cell reproduces zero;
// lanes past the grid edge only have to skip their loads and stores.
#include "common.h"

namespace rtm {
namespace {

constexpr float kC1 = 1.6f;
constexpr float kC2 = -0.2f;
constexpr float kC3 = 8.0f / 315.0f;
constexpr float kC4 = -1.0f / 560.0f;

__device__ __forceinline__ float dpp_shr1(float old, float src)
{
    // wave_shr:1 - lane i receives lane i-1; lane 0 keeps `old`.
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), 0x138, 0xf,
                                                      0xf, false));
}

__device__ __forceinline__ float dpp_shl1(float old, float src)
{
    // wave_shl:1 - lane i receives lane i+1; lane 63 keeps `old`.
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), 0x130, 0xf,
                                                      0xf, false));
}

template <int VEC>
__device__ __forceinline__ void ldv(const float *p, float (&v)[VEC])
{
    if constexpr (VEC == 4) {
        float4 t = *reinterpret_cast<const float4 *>(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (VEC == 2) {
        float2 t = *reinterpret_cast<const float2 *>(p);
        v[0] = t.x; v[1] = t.y;
    } else {
        v[0] = *p;
    }
}

template <int VEC>
__device__ __forceinline__ void stv(float *p, const float (&v)[VEC])
{
    if constexpr (VEC == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (VEC == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
    } else {
        *p = v[0];
    }
}

// Unscaled 8th-order second difference along one direction from the
// neighbours at -4..4 (a[4] is the centre), in difference form.
__device__ __forceinline__ float d2_diff(float c, float m1, float p1, float m2, float p2, float m3, float p3,
                                         float m4, float p4)
{
    float s = kC1 * ((p1 - c) + (m1 - c));
    s = fmaf(kC2, (p2 - c) + (m2 - c), s);
    s = fmaf(kC3, (p3 - c) + (m3 - c), s);
    s = fmaf(kC4, (p4 - c) + (m4 - c), s);
    return s;
}

// Row of 4 + VEC + 4 values around the lane's VEC centre cells, built from
// the neighbouring lanes by DPP shifts.  hl / hr are the halo floats at the
// strip ends (meaningful in lanes 0 and 63 only).
template <int VEC>
__device__ __forceinline__ void exchange_row(const float (&c)[VEC], const float (&hl)[4], const float (&hr)[4],
                                             float (&ext)[VEC + 8])
{
    constexpr int K = 4 / VEC;
#pragma unroll
    for (int j = 0; j < VEC; ++j) ext[4 + j] = c[j];
    float L[VEC], Rr[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        L[j] = c[j];
        Rr[j] = c[j];
    }
#pragma unroll
    for (int k = 1; k <= K; ++k) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            L[j] = dpp_shr1(hl[4 - k * VEC + j], L[j]);
            Rr[j] = dpp_shl1(hr[(k - 1) * VEC + j], Rr[j]);
            ext[4 - k * VEC + j] = L[j];
            ext[4 + VEC + (k - 1) * VEC + j] = Rr[j];
        }
    }
}

// Loads the strip-end halo of one row: lane 0 the 4 cells left of the
// strip, lane 63 the 4 cells right of it (zeros past the stored columns).
template <int VEC>
__device__ __forceinline__ void load_halo(const float *row, int x0, int NX, int lane, float (&hl)[4], float (&hr)[4])
{
    hl[0] = hl[1] = hl[2] = hl[3] = 0.f;
    hr[0] = hr[1] = hr[2] = hr[3] = 0.f;
    if (lane == 0) {
        float4 t = *reinterpret_cast<const float4 *>(row + x0 - 4);
        hl[0] = t.x; hl[1] = t.y; hl[2] = t.z; hl[3] = t.w;
    } else if (lane == 63) {
        int xr = x0 + 64 * VEC;
        if (xr < NX + kRadius) {
            float4 t = *reinterpret_cast<const float4 *>(row + xr);
            hr[0] = t.x; hr[1] = t.y; hr[2] = t.z; hr[3] = t.w;
        }
    }
}

// Weighted signal sum of the injection nodes of this lane's cells in row z.
// `e` walks the row-sorted entries [e, eend); `sig` is indexed by each
// contribution's signal index.  Adds into add[0..VEC).
template <int VEC>
__device__ __forceinline__ void gather_inj(int &e, int eend, int z, int x, const InjEnt *__restrict__ ents,
                                           const Contrib *__restrict__ cont, const float *__restrict__ sig,
                                           float (&add)[VEC])
{
    while (e < eend && ents[e].z == z) {
        const InjEnt E = ents[e];
        int j = E.x - x;
        if (j >= 0 && j < VEC) {
            float s = 0.f;
            for (int c = E.cbeg; c < E.cend; ++c) s = fmaf(cont[c].w, sig[cont[c].idx], s);
#pragma unroll
            for (int jj = 0; jj < VEC; ++jj)
                if (jj == j) add[jj] += s;
        }
        ++e;
    }
}

// Receivers [r0, r0 + 64) of one shot: d[n][r] = sum_q w_q p^n[node_q].
__device__ __forceinline__ void sample_body(const ShotDev *__restrict__ shots, SampleTask task, int n)
{
    const ShotDev &S = shots[task.shot];
    int r = task.r0 + (int)threadIdx.x;
    if (r >= S.nrec) return;
    const float *p = S.fld[n & 1] + S.L.org;
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kMaxNodes; ++q) {
        float w = S.rw[r * kMaxNodes + q];
        int off = S.rnode[r * kMaxNodes + q];
        s = fmaf(w, p[off], s);
    }
    S.rec_out[(int64_t)n * S.nrec + r] = s;
}

}  // namespace

// Forward step n of every tile:  p^{n+1} = 2 p^n - p^{n-1} + D' (L p^n + s^n),
// written over p^{n-1}; workgroups past the stencil slots record d^n = R p^n.
template <int VEC>
__global__ __launch_bounds__(64) void fwd2d_kernel(const ShotDev *__restrict__ shots,
                                                   const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                                                   const InjEnt *__restrict__ ents,
                                                   const Contrib *__restrict__ cont,
                                                   const SampleTask *__restrict__ stasks, int n)
{
    const int lane = threadIdx.x;
    const int b = blockIdx.x;
    if (b >= nslots) {
        sample_body(shots, stasks[b - nslots], n);
        return;
    }
    const int t = xcd_tile(b, nslots);
    if (t >= ntiles) return;
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const int64_t pitch = S.L.pitch;
    const int NX = S.L.NX;
    const float *__restrict__ pc = S.fld[n & 1] + S.L.org;
    float *__restrict__ po = S.fld[(n + 1) & 1] + S.L.org;
    const float *__restrict__ Dp = S.Dp + S.L.org;
    const float *__restrict__ wav = S.wav + n;

    const int x = T.x0 + lane * VEC;
    const bool live = x < NX + kRadius;
    const bool own = x < NX;

    float q[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) q[i][j] = 0.f;
        if (live) ldv<VEC>(pc + (int64_t)(T.z0 - 4 + i) * pitch + x, q[i]);
    }
    int es = T.sbeg;
    for (int z = T.z0; z < T.z1; ++z) {
        const float *row = pc + (int64_t)z * pitch;
#pragma unroll
        for (int j = 0; j < VEC; ++j) q[8][j] = 0.f;
        float old[VEC], d[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) old[j] = d[j] = 0.f;
        if (live) {
            ldv<VEC>(pc + (int64_t)(z + 4) * pitch + x, q[8]);
            ldv<VEC>(po + (int64_t)z * pitch + x, old);
            ldv<VEC>(Dp + (int64_t)z * pitch + x, d);
        }
        float hl[4], hr[4];
        load_halo<VEC>(row, T.x0, NX, lane, hl, hr);
        float ext[VEC + 8];
        exchange_row<VEC>(q[4], hl, hr, ext);
        float add[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) add[j] = 0.f;
        gather_inj<VEC>(es, T.send, z, x, ents, cont, wav, add);
        float out[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = q[4][j];
            float lap = d2_diff(c, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j],
                                ext[8 + j]);
            lap += d2_diff(c, q[3][j], q[5][j], q[2][j], q[6][j], q[1][j], q[7][j], q[0][j], q[8][j]);
            out[j] = fmaf(d[j], lap + add[j], 2.f * c - old[j]);
        }
        if (own) stv<VEC>(po + (int64_t)z * pitch + x, out);
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < VEC; ++j) q[i][j] = q[i + 1][j];
    }
}

// Reverse step k of every tile, Eqs. (2), (3) and (6) in one pass:
//   p^{k-1} = 2 p^k - p^{k+1} + D' (L p^k + s^k)         (reconstruction)
//   mu^k    = 2 mu^{k+1} - mu^{k+2} + D' (L mu^{k+1} + r^k)  (receiver field)
// and either the imaging sums num += p^k mu^{k+1}, den += (p^k)^2 on the
// interior (GRAD = false) or the gradient sum G += mu^{k+1} D' (L p^k + s^k)
// on the whole padded grid (GRAD = true).  With reinject = 0 the source term
// is left out of the reconstruction (Eq. (6) as written).  When wadj is
// non-null, the lane owning each source node writes its coefficient times
// mu^{k+1} to wadj[k * kMaxNodes + node] for the wavelet adjoint.
template <int VEC, bool GRAD>
__global__ __launch_bounds__(64) void rev2d_kernel(const ShotDev *__restrict__ shots,
                                                   const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                                                   const InjEnt *__restrict__ ents,
                                                   const Contrib *__restrict__ cont, int k, int reinject,
                                                   float *__restrict__ wadj)
{
    const int lane = threadIdx.x;
    const int t = xcd_tile(blockIdx.x, nslots);
    if (t >= ntiles) return;
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    const int64_t pitch = S.L.pitch;
    const int NX = S.L.NX;
    const float *__restrict__ P0 = S.fld[k & 1] + S.L.org;            // p^k
    float *__restrict__ P1 = S.fld[(k + 1) & 1] + S.L.org;            // p^{k+1} -> p^{k-1}
    const float *__restrict__ M0 = S.fld[2 + ((k + 1) & 1)] + S.L.org;  // mu^{k+1}
    float *__restrict__ M1 = S.fld[2 + (k & 1)] + S.L.org;            // mu^{k+2} -> mu^k
    const float *__restrict__ Dp = S.Dp + S.L.org;
    float *__restrict__ A0 = S.acc0 + S.L.org;
    float *__restrict__ A1 = GRAD ? nullptr : S.acc1 + S.L.org;
    const float *__restrict__ wav = S.wav + k;
    const float *__restrict__ sig = S.sig + (int64_t)k * S.nrec;

    const int x = T.x0 + lane * VEC;
    const bool live = x < NX + kRadius;
    const bool own = x < NX;
    // Lanes whose cells overlap the interior accumulate the image sums (their
    // other cells lie in the band or halo, whose sums are never read).
    const bool own_img = own && x + VEC > S.ix0 && x < S.ix1;

    float qp[9][VEC], qm[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) qp[i][j] = qm[i][j] = 0.f;
        if (live) {
            ldv<VEC>(P0 + (int64_t)(T.z0 - 4 + i) * pitch + x, qp[i]);
            ldv<VEC>(M0 + (int64_t)(T.z0 - 4 + i) * pitch + x, qm[i]);
        }
    }
    int es = T.sbeg, er = T.rbeg;
    for (int z = T.z0; z < T.z1; ++z) {
        const int64_t o = (int64_t)z * pitch + x;
#pragma unroll
        for (int j = 0; j < VEC; ++j) qp[8][j] = qm[8][j] = 0.f;
        float p1[VEC], m1[VEC], d[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) p1[j] = m1[j] = d[j] = 0.f;
        if (live) {
            ldv<VEC>(P0 + o + 4 * pitch, qp[8]);
            ldv<VEC>(M0 + o + 4 * pitch, qm[8]);
            ldv<VEC>(P1 + o, p1);
            ldv<VEC>(M1 + o, m1);
            ldv<VEC>(Dp + o, d);
        }
        float hl[4], hr[4], ext_p[VEC + 8], ext_m[VEC + 8];
        load_halo<VEC>(P0 + (int64_t)z * pitch, T.x0, NX, lane, hl, hr);
        exchange_row<VEC>(qp[4], hl, hr, ext_p);
        load_halo<VEC>(M0 + (int64_t)z * pitch, T.x0, NX, lane, hl, hr);
        exchange_row<VEC>(qm[4], hl, hr, ext_m);

        float sadd[VEC], radd[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) sadd[j] = radd[j] = 0.f;
        if (wadj) {
            // Source nodes of this row: record coefficient * mu^{k+1}.
            while (es < T.send && ents[es].z == z) {
                const InjEnt E = ents[es];
                int j = E.x - x;
                if (j >= 0 && j < VEC) {
                    float s = 0.f, mval = 0.f;
                    for (int c = E.cbeg; c < E.cend; ++c) s = fmaf(cont[c].w, wav[0], s);
#pragma unroll
                    for (int jj = 0; jj < VEC; ++jj)
                        if (jj == j) {
                            sadd[jj] += s;
                            mval = qm[4][jj];
                        }
                    float wsum = 0.f;
                    for (int c = E.cbeg; c < E.cend; ++c) wsum += cont[c].w;
                    wadj[(int64_t)k * kMaxNodes + E.slot] = wsum * mval;
                }
                ++es;
            }
        } else {
            gather_inj<VEC>(es, T.send, z, x, ents, cont, wav, sadd);
        }
        gather_inj<VEC>(er, T.rend, z, x, ents, cont, sig, radd);

        float np[VEC], nm[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const float c = qp[4][j];
            float lap = d2_diff(c, ext_p[3 + j], ext_p[5 + j], ext_p[2 + j], ext_p[6 + j], ext_p[1 + j],
                                ext_p[7 + j], ext_p[j], ext_p[8 + j]);
            lap += d2_diff(c, qp[3][j], qp[5][j], qp[2][j], qp[6][j], qp[1][j], qp[7][j], qp[0][j], qp[8][j]);
            const float inc = d[j] * (lap + sadd[j]);
            np[j] = (reinject ? inc : d[j] * lap) + (2.f * c - p1[j]);
            const float cm = qm[4][j];
            float lapm = d2_diff(cm, ext_m[3 + j], ext_m[5 + j], ext_m[2 + j], ext_m[6 + j], ext_m[1 + j],
                                 ext_m[7 + j], ext_m[j], ext_m[8 + j]);
            lapm += d2_diff(cm, qm[3][j], qm[5][j], qm[2][j], qm[6][j], qm[1][j], qm[7][j], qm[0][j], qm[8][j]);
            nm[j] = fmaf(d[j], lapm + radd[j], 2.f * cm - m1[j]);
            if (GRAD) sadd[j] = inc;  // reuse: second time difference of p at step k
        }
        if (own) {
            stv<VEC>(P1 + o, np);
            stv<VEC>(M1 + o, nm);
        }
        if (GRAD) {
            if (own) {
                float g[VEC];
                ldv<VEC>(A0 + o, g);
#pragma unroll
                for (int j = 0; j < VEC; ++j) g[j] = fmaf(qm[4][j], sadd[j], g[j]);
                stv<VEC>(A0 + o, g);
            }
        } else if (z >= S.iz0 && z < S.iz1 && own_img) {
            float a[VEC], bb[VEC];
            ldv<VEC>(A0 + o, a);
            ldv<VEC>(A1 + o, bb);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                a[j] = fmaf(qp[4][j], qm[4][j], a[j]);
                bb[j] = fmaf(qp[4][j], qp[4][j], bb[j]);
            }
            stv<VEC>(A0 + o, a);
            stv<VEC>(A1 + o, bb);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                qp[i][j] = qp[i + 1][j];
                qm[i][j] = qm[i + 1][j];
            }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

hipError_t launch_fwd2d(int vec, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, const SampleTask *stasks, int nsample, int n,
                        hipStream_t st)
{
    dim3 grid(nslots + nsample), block(64);
    switch (vec) {
    case 1: hipLaunchKernelGGL(fwd2d_kernel<1>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, n); break;
    case 2: hipLaunchKernelGGL(fwd2d_kernel<2>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, n); break;
    case 4: hipLaunchKernelGGL(fwd2d_kernel<4>, grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, stasks, n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rev2d(int vec, bool grad, const ShotDev *shots, const Tile2D *tiles, int ntiles, int nslots,
                        const InjEnt *ents, const Contrib *cont, int k, int reinject, float *wadj, hipStream_t st)
{
    dim3 grid(nslots), block(64);
#define RTM_REV2D(V, G) \
    hipLaunchKernelGGL((rev2d_kernel<V, G>), grid, block, 0, st, shots, tiles, ntiles, nslots, ents, cont, k, reinject, wadj)
    if (grad) {
        switch (vec) {
        case 1: RTM_REV2D(1, true); break;
        case 2: RTM_REV2D(2, true); break;
        case 4: RTM_REV2D(4, true); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (vec) {
        case 1: RTM_REV2D(1, false); break;
        case 2: RTM_REV2D(2, false); break;
        case 4: RTM_REV2D(4, false); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef RTM_REV2D
    return hipGetLastError();
}

}  // namespace rtm

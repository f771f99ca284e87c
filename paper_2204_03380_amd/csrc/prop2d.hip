// 2-D propagation kernels for gfx950.
//
// One wavefront (64 lanes) owns a strip of 64 * VEC consecutive x cells and
// marches down the rows [z0, z1) of its tile.  Each lane keeps the nine rows
// z-4 .. z+4 of its VEC cells in registers (a register queue), so every
// stored value of the input field is read from memory once per tile plus the
// 8-row overlap with the tiles above and below.  The march is unrolled by
// nine so that the queue rotates by register renaming, not by moves.  The
// x-neighbours of the centre row come from the adjacent lanes through DPP
// wave shifts; lanes 0 and 63 supply the 4-cell halo at the strip ends with
// one extra load.
//
// The stencil is evaluated as
//   L p_i = sum_axis sum_{m=1..4} c_m ((p_{i+m} + p_{i-m}) - 2 p_i),
// algebraically the 8th-order Laplacian of Sec. 3, but exactly zero on a
// constant field in FP32: the rounded weights then cannot add a spurious
// mass term, which would otherwise accumulate into a phase error of ~1e-3
// after a few thousand steps.
//
// Fields are stored with a zero halo and the scaled velocity term
// D' = (v dt / h)^2 is zero there, so updating a halo cell reproduces zero;
// lanes past the grid edge only have to skip their loads and stores.
#include "stencil.h"

namespace rtm {
namespace {

// --------------------------------------------------------------------------
// Forward step
// --------------------------------------------------------------------------

template <int VEC>
struct FwdCtx {
    const gfloat *pc;  // p^n
    gfloat *po;        // p^{n-1}, overwritten by p^{n+1}
    const gfloat *Dp;
    int64_t pitch;
    int x, x0, NX, lane;
    bool live, own;
};

// Row z of the march.  Queue slot (S + i) % 9 holds row z - 4 + i; the slot
// of row z + 4 is refilled here.
template <int VEC, int S>
__device__ __forceinline__ void fwd_row(const FwdCtx<VEC> &C, float (&q)[9][VEC], int z)
{
    constexpr int r0 = (S + 0) % 9, r1 = (S + 1) % 9, r2 = (S + 2) % 9, r3 = (S + 3) % 9, r4 = (S + 4) % 9,
                  r5 = (S + 5) % 9, r6 = (S + 6) % 9, r7 = (S + 7) % 9, r8 = (S + 8) % 9;
    const int64_t o = (int64_t)z * C.pitch + C.x;
    float old[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) q[r8][j] = old[j] = d[j] = 0.f;
    if (C.live) {
        ldv<VEC>(C.pc + o + 4 * C.pitch, q[r8]);
        ldv<VEC>(C.po + o, old);
        ldv<VEC>(C.Dp + o, d);
    }
    float hl[4], hr[4], ext[VEC + 8];
    load_halo<VEC>(C.pc + (int64_t)z * C.pitch, C.x0, C.NX, C.lane, hl, hr);
    exchange_row<VEC>(q[r4], hl, hr, ext);
    float out[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = q[r4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, q[r3][j], q[r5][j], q[r2][j], q[r6][j], q[r1][j], q[r7][j], q[r0][j], q[r8][j]);
        out[j] = fmaf(d[j], lap, c2 - old[j]);
    }
    if (C.own) stv<VEC>(C.po + o, out);
}

// --------------------------------------------------------------------------
// Reverse step
// --------------------------------------------------------------------------

template <int VEC>
struct RevCtx {
    const gfloat *P0;  // p^k
    gfloat *P1;        // p^{k+1} -> p^{k-1}
    const gfloat *M0;  // mu^{k+1}
    gfloat *M1;        // mu^{k+2} -> mu^k
    const gfloat *Dp;
    gfloat *A0, *A1;   // num, den | G
    int64_t pitch;
    int x, x0, NX, lane, iz0, iz1;
    bool live, own, own_img, reinject;
};

template <int VEC, bool GRAD, int S>
__device__ __forceinline__ void rev_row(const RevCtx<VEC> &C, float (&qp)[9][VEC], float (&qm)[9][VEC], int z)
{
    constexpr int r0 = (S + 0) % 9, r1 = (S + 1) % 9, r2 = (S + 2) % 9, r3 = (S + 3) % 9, r4 = (S + 4) % 9,
                  r5 = (S + 5) % 9, r6 = (S + 6) % 9, r7 = (S + 7) % 9, r8 = (S + 8) % 9;
    const int64_t o = (int64_t)z * C.pitch + C.x;
    float p1[VEC], m1[VEC], d[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) qp[r8][j] = qm[r8][j] = p1[j] = m1[j] = d[j] = 0.f;
    if (C.live) {
        ldv<VEC>(C.P0 + o + 4 * C.pitch, qp[r8]);
        ldv<VEC>(C.M0 + o + 4 * C.pitch, qm[r8]);
        ldv_s<VEC>(C.P1 + o, p1);
        ldv_s<VEC>(C.M1 + o, m1);
        ldv_s<VEC>(C.Dp + o, d);
    }
    float hl[4], hr[4], ext[VEC + 8];
    float np[VEC], nm[VEC], inc[VEC];
    load_halo<VEC>(C.P0 + (int64_t)z * C.pitch, C.x0, C.NX, C.lane, hl, hr);
    exchange_row<VEC>(qp[r4], hl, hr, ext);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = qp[r4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, qp[r3][j], qp[r5][j], qp[r2][j], qp[r6][j], qp[r1][j], qp[r7][j], qp[r0][j], qp[r8][j]);
        inc[j] = d[j] * lap;
        np[j] = inc[j] + (c2 - p1[j]);
    }
    if (C.own) stv<VEC>(C.P1 + o, np);
    load_halo<VEC>(C.M0 + (int64_t)z * C.pitch, C.x0, C.NX, C.lane, hl, hr);
    exchange_row<VEC>(qm[r4], hl, hr, ext);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float c = qm[r4][j], c2 = c + c;
        float lap = d2(c2, ext[3 + j], ext[5 + j], ext[2 + j], ext[6 + j], ext[1 + j], ext[7 + j], ext[j], ext[8 + j]);
        lap += d2(c2, qm[r3][j], qm[r5][j], qm[r2][j], qm[r6][j], qm[r1][j], qm[r7][j], qm[r0][j], qm[r8][j]);
        nm[j] = fmaf(d[j], lap, c2 - m1[j]);
    }
    if (C.own) stv<VEC>(C.M1 + o, nm);
    if constexpr (GRAD) {
        if (C.own) {
            float g[VEC];
            ldv<VEC>(C.A0 + o, g);
#pragma unroll
            for (int j = 0; j < VEC; ++j) g[j] = fmaf(qm[r4][j], inc[j], g[j]);
            stv<VEC>(C.A0 + o, g);
        }
    } else {
        if (z >= C.iz0 && z < C.iz1 && C.own_img) {
            float a[VEC], b[VEC];
            ldv_s<VEC>(C.A0 + o, a);
            ldv_s<VEC>(C.A1 + o, b);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                a[j] = fmaf(qp[r4][j], qm[r4][j], a[j]);
                b[j] = fmaf(qp[r4][j], qp[r4][j], b[j]);
            }
            stv_s<VEC>(C.A0 + o, a);
            stv_s<VEC>(C.A1 + o, b);
        }
    }
}

// Runs ROWCALL(S, z) over the tile's rows, nine per trip (z1 - z0 is a
// multiple of nine), so that S = (z - z0) mod 9 is a compile-time constant.
#define RTM_MARCH(ROWCALL)                                                                     \
    for (int z = T.z0; z < T.z1; z += kZUnroll) {                                              \
        ROWCALL(0, z); ROWCALL(1, z + 1); ROWCALL(2, z + 2); ROWCALL(3, z + 3);                \
        ROWCALL(4, z + 4); ROWCALL(5, z + 5); ROWCALL(6, z + 6); ROWCALL(7, z + 7);            \
        ROWCALL(8, z + 8);                                                                     \
    }

}  // namespace

// Forward step n of every tile:  p^{n+1} = 2 p^n - p^{n-1} + D' (L p^n + s^n),
// written over p^{n-1}; workgroups past the stencil slots record d^n = R p^n.
// The source term is added to the stored value after the march by the lane
// that stored it (same thread, so program order makes the value visible).
template <int VEC>
__global__ __launch_bounds__(64) void fwd2d_kernel(const ShotDev *__restrict__ shots,
                                                   const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                                                   const InjEnt *__restrict__ ents,
                                                   const Contrib *__restrict__ cont,
                                                   const SampleTask *__restrict__ stasks, int n)
{
    const int b = blockIdx.x;
    if (b >= nslots) {
        sample_body(shots, stasks[b - nslots], n, (int)threadIdx.x);
        return;
    }
    const int t = xcd_tile(b, nslots);
    if (t >= ntiles) return;
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    FwdCtx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.pc = gp(S.fld[n & 1] + S.L.org);
    C.po = gp(S.fld[(n + 1) & 1] + S.L.org);
    C.Dp = gp(S.Dp + S.L.org);
    C.lane = threadIdx.x;
    C.x0 = T.x0;
    C.x = T.x0 + C.lane * VEC;
    C.live = C.x < C.NX + kRadius;
    C.own = C.x < C.NX;

    float q[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) q[i][j] = 0.f;
        if (C.live) ldv<VEC>(C.pc + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, q[i]);
    }
#define RTM_FWD_ROW(SS, ZZ) fwd_row<VEC, SS>(C, q, ZZ)
    RTM_MARCH(RTM_FWD_ROW)
#undef RTM_FWD_ROW
    // Source injection: p^{n+1} += D' s^n at the source nodes of this tile.
    const float *wav = S.wav + n;
    for (int e = T.sbeg; e < T.send; ++e) {
        const InjEnt E = ents[e];
        if (owns<VEC>(E.x, T.x0, C.lane)) {
            const int64_t o = (int64_t)E.z * C.pitch + E.x;
            C.po[o] = fmaf(C.Dp[o], inj_sum(E, cont, wav), C.po[o]);
        }
    }
}

// Reverse step k of every tile, Eqs. (2), (3) and (6) in one pass:
//   p^{k-1} = 2 p^k - p^{k+1} + D' (L p^k + s^k)         (reconstruction)
//   mu^k    = 2 mu^{k+1} - mu^{k+2} + D' (L mu^{k+1} + r^k)  (receiver field)
// and either the imaging sums num += p^k mu^{k+1}, den += (p^k)^2 on the
// interior (GRAD = false) or the gradient sum G += mu^{k+1} D' (L p^k + s^k)
// on the whole padded grid (GRAD = true).  With reinject = 0 the source term
// is left out of the reconstruction (Eq. (6) as written).  The source and
// receiver terms are added after the march by the lanes that stored the
// cells.  When wadj is non-null, those lanes also write each source node's
// coefficient times mu^{k+1} to wadj[k * kMaxNodes + node].
// With one float per lane the reverse kernel fits in 64 registers; asking
// for 8 waves per SIMD then hides more latency (measured: 4.5 vs 4.2 TB/s
// on 16 shots of the 2301 x 751 grid).  Wider lanes would spill.
template <int VEC, bool GRAD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(VEC == 1 ? 8 : 1, 8)))
void rev2d_kernel(const ShotDev *__restrict__ shots,
                                                   const Tile2D *__restrict__ tiles, int ntiles, int nslots,
                                                   const InjEnt *__restrict__ ents,
                                                   const Contrib *__restrict__ cont, int k, int reinject,
                                                   float *__restrict__ wadj)
{
    const int t = xcd_tile(blockIdx.x, nslots);
    if (t >= ntiles) return;
    const Tile2D T = tiles[t];
    const ShotDev &S = shots[T.shot];
    RevCtx<VEC> C;
    C.pitch = S.L.pitch;
    C.NX = S.L.NX;
    C.P0 = gp(S.fld[k & 1] + S.L.org);
    C.P1 = gp(S.fld[(k + 1) & 1] + S.L.org);
    C.M0 = gp(S.fld[2 + ((k + 1) & 1)] + S.L.org);
    C.M1 = gp(S.fld[2 + (k & 1)] + S.L.org);
    C.Dp = gp(S.Dp + S.L.org);
    C.A0 = gp(S.acc0 + S.L.org);
    C.A1 = GRAD ? nullptr : gp(S.acc1 + S.L.org);
    C.lane = threadIdx.x;
    C.x0 = T.x0;
    C.x = T.x0 + C.lane * VEC;
    C.live = C.x < C.NX + kRadius;
    C.own = C.x < C.NX;
    // Lanes whose cells overlap the interior accumulate the image sums (their
    // other cells lie in the band or halo, whose sums are never read).
    C.own_img = C.own && C.x + VEC > S.ix0 && C.x < S.ix1;
    C.iz0 = S.iz0;
    C.iz1 = S.iz1;
    C.reinject = reinject != 0;

    float qp[9][VEC], qm[9][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) qp[i][j] = qm[i][j] = 0.f;
        if (C.live) {
            ldv<VEC>(C.P0 + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, qp[i]);
            ldv<VEC>(C.M0 + (int64_t)(T.z0 - 4 + i) * C.pitch + C.x, qm[i]);
        }
    }
#define RTM_REV_ROW(SS, ZZ) rev_row<VEC, GRAD, SS>(C, qp, qm, ZZ)
    RTM_MARCH(RTM_REV_ROW)
#undef RTM_REV_ROW
    // Source term at step k: reconstruction (re-injection), gradient, wavelet adjoint.
    const float *wav = S.wav + k;
    for (int e = T.sbeg; e < T.send; ++e) {
        const InjEnt E = ents[e];
        if (owns<VEC>(E.x, T.x0, C.lane)) {
            const int64_t o = (int64_t)E.z * C.pitch + E.x;
            const float ds = C.Dp[o] * inj_sum(E, cont, wav);
            if (C.reinject) C.P1[o] = C.P1[o] + ds;
            if (GRAD) C.A0[o] = fmaf(C.M0[o], ds, C.A0[o]);
            if (wadj) {
                float wsum = 0.f;
                for (int c = E.cbeg; c < E.cend; ++c) wsum += cont[c].w;
                wadj[(int64_t)k * kMaxNodes + E.slot] = wsum * C.M0[o];
            }
        }
    }
    // Receiver term: mu^k += D' R^T g^k.
    const float *sig = S.sig + (int64_t)k * S.nrec;
    for (int e = T.rbeg; e < T.rend; ++e) {
        const InjEnt E = ents[e];
        if (owns<VEC>(E.x, T.x0, C.lane)) {
            const int64_t o = (int64_t)E.z * C.pitch + E.x;
            C.M1[o] = fmaf(C.Dp[o], inj_sum(E, cont, sig), C.M1[o]);
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

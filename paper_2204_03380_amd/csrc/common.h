// Internal definitions shared by the host runtime and the HIP kernels of
// librtm.  Not part of the public ABI (include/rtm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtm {

// Stencil radius of the 8th-order second derivative.
constexpr int kRadius = 4;
// Column of interior-padded cell x = 0 inside a stored row.  32 floats keep
// every strip start on a 128-byte line and leave room for the 4-cell halo.
constexpr int kXOff = 32;
// Maximum interpolation nodes of a point (multilinear: 2^ndim).
constexpr int kMaxNodes = 8;
// Number of XCDs on MI355X; workgroups are dispatched to them round robin.
constexpr int kNumXcd = 8;

// Tiles march down z in groups of kZUnroll rows (the length of the register
// queue), so the stored rows are rounded up to a multiple of it.
constexpr int kZUnroll = 9;

// Storage of one wavefield-sized array with a zero halo of kRadius cells on
// every side of the padded grid (and, below it, up to kZUnroll - 1 further
// zero rows so that every tile marches a multiple of kZUnroll rows).  Cell
// (z, y, x) of the padded grid lives at org + z * plane + y * pitch + x.
struct Layout {
    int NX, NY, NZ;   // padded extents (NY = 1 in 2-D)
    int NZr;          // NZ rounded up to a multiple of kZUnroll
    int ndim;
    int64_t pitch;    // floats per stored row
    int64_t plane;    // floats per stored z-plane (== pitch in 2-D)
    int64_t org;      // index of padded cell (0, 0, 0)
    int64_t total;    // floats per array, halo included
};

inline Layout make_layout(int ndim, int NX, int NY, int NZ)
{
    Layout L;
    L.ndim = ndim;
    L.NX = NX;
    L.NY = (ndim == 3) ? NY : 1;
    L.NZ = NZ;
    L.NZr = (NZ + kZUnroll - 1) / kZUnroll * kZUnroll;
    // Loads reach column kXOff + NX + 6 at most: a lane starting at or below
    // cell NX + 3 reads up to 4 floats, and the right strip halo likewise.
    int64_t row = kXOff + NX + 2 * kRadius;
    L.pitch = (row + 63) / 64 * 64;
    if (ndim == 3) {
        L.plane = (int64_t)(L.NY + 2 * kRadius) * L.pitch;
        L.org = kRadius * L.plane + kRadius * L.pitch + kXOff;
    } else {
        L.plane = L.pitch;
        L.org = kRadius * L.pitch + kXOff;
    }
    L.total = (int64_t)(L.NZr + 2 * kRadius) * L.plane;
    return L;
}

// Per-shot state seen by the propagation kernels.  Wavefields are
// addressed through `fld`: p^m lives in fld[m & 1] and the receiver
// wavefield mu^m in fld[2 + (m & 1)].  fld[4 .. 7] (2-D jobs) are a second
// set with the same roles: a two-step launch reads the first set and writes
// the second, and the host then swaps to a copy of the shot table whose two
// sets are exchanged, so every kernel keeps addressing the current levels
// through fld[0 .. 3].
struct ShotDev {
    float *fld[8];
    float *acc0;        // num (imaging) or G (gradient)
    float *acc1;        // den (imaging) or unused
    const float *Dp;    // (v dt / h)^2, zero in the halo
    const float *wav;   // wavelet [nt]
    const float *sig;   // receiver signal [nt + 1][nrec] (reverse passes)
    float *rec_out;     // recorded samples [nt + 1][nrec] (forward pass)
    const int *rnode;   // [nrec][kMaxNodes] node offsets from cell (0,0,0)
    const float *rw;    // [nrec][kMaxNodes] interpolation weights (0 = unused)
    int nrec;
    int ix0, ix1, iy0, iy1, iz0, iz1;  // interior box, padded coordinates [lo, hi)
    int sz0, sz1;       // padded rows [sz0, sz1) holding receiver nodes (2-D)
    Layout L;
};

// A 2-D stencil tile: one wavefront marches down rows [z0, z1) of a strip
// of 64 * VEC columns starting at x0; z1 - z0 is a multiple of kZUnroll
// (rows at or below NZ are zero halo rows and stay zero).  Injection entries
// of the tile are ents[sbeg, send) (source, into p) and ents[rbeg, rend)
// (receivers, into mu).  A tile of T > 1 steps per launch also lists the
// entries of its whole strip and rows [z0 - 4 (T - 1), z1 + 4 (T - 1)) (where
// the first step is computed) in ents[s1beg, s1end) and ents[r1beg, r1end),
// and with T = 3 those of rows [z0 - 4, z1 + 4) (where the second step is
// computed) in ents[s2beg, s2end) and ents[r2beg, r2end).  The tile's own
// list (sbeg .. rend) feeds the last step.
struct Tile2D {
    int shot;
    int x0, z0, z1;
    int sbeg, send, rbeg, rend;
    int s1beg, s1end, r1beg, r1end;
    int s2beg, s2end, r2beg, r2end;
};

// A 3-D stencil tile: a workgroup covers x in [x0, x0 + TX) and y in
// [y0, y0 + TY) and marches z over [z0, z1).
struct Tile3D {
    int shot;
    int x0, y0, z0, z1;
    int sbeg, send, rbeg, rend;
};

// One injection node: padded coordinates and the contributions
// cont[cbeg, cend) whose weighted signal sum is added at the node.  `slot`
// numbers the nodes of the source point (0 .. 2^ndim - 1), for the wavelet
// adjoint; `shot` is the owning shot.
struct InjEnt {
    int z, y, x;
    int cbeg, cend;
    int slot;
    int shot;
    int pad_;
};

// Contribution to an injection node: signal index (receiver number, or 0
// for the wavelet) and its weight (interpolation weight times h-scaling).
struct Contrib {
    int idx;
    float w;
};

// Sampling work item: receivers [r0, r0 + 64) of one shot.
struct SampleTask {
    int shot;
    int r0;
};

// Work item of a persistent pass (one launch for all time steps): a tile
// (idx >= 0) or a receiver sampling task (idx = -1 - task) of shot `shot`.
// Each item of a shot waits, at time step r of the pass, until the shot's
// counter shows all of the shot's items of step r - 1 done.
struct PItem {
    int idx;
    int shot;
};

// Band options of the random-boundary padding (Eqs. (4)-(5) taper, free
// surface): passed to the padding kernels by value.
constexpr int kMaxTaper = 256;
constexpr unsigned kBandTaper = 0x1u;
constexpr unsigned kBandFreeSurface = 0x2u;
struct BandOpts {
    unsigned flags;
    float c[kMaxTaper];  // taper coefficient of band depth i at c[i - 1]
};

// Map a workgroup index onto a tile index so that each XCD processes a
// contiguous range of tiles (neighbouring tiles share halo rows in that
// XCD's L2).  `nslots` is a multiple of kNumXcd; slot values >= ntiles are
// idle.  The map is a bijection on [0, nslots).
__host__ __device__ inline int xcd_tile(int b, int nslots)
{
    int per = nslots / kNumXcd;
    return (b % kNumXcd) * per + b / kNumXcd;
}

}  // namespace rtm

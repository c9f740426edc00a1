// Row layout helpers shared by the two-buffer and in-place row kernels.
//
// Row layout: the 19 populations of lattice row r = y + ny z are 19
// consecutive runs of nx values, population a of node x at element
// (19 r + a) nx + x (Geom::plane = nx, Geom::row = 19 nx).  A row kernel
// runs waves of 64 consecutive x of one row (blockDim.x a multiple of 64),
// so every direction's source or target run has a uniform (scalar) base and
// one lane offset serves all of them.  Rows off the y and z faces and rows on
// them go to separate launches: the inner-row kernels then carry no face
// logic.
#pragma once

#include "clbm_internal.hpp"

namespace clbm {

__device__ inline __amdgpu_buffer_rsrc_t row_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferFlags);
}

struct RowGrid {
    uint32_t gx;            // tiles along x
    uint32_t rows;          // rows handled by the launch
    uint32_t aligned;       // largest multiple of 8 <= number of workgroups
    int32_t remap;          // XCD-contiguous tile order
    int32_t zf, yf;         // face rows: z faces (1 or 2) and y faces (1 or 2)
};

// Row index of the wave and tile of the workgroup (blockDim.x a multiple of 64).
__device__ inline bool row_of(const RowGrid &R, int &x, uint32_t &ri) {
    uint32_t b = blockIdx.x;
    if (R.remap && b < R.aligned) b = (b & 7u) * (R.aligned >> 3) + (b >> 3);
    const uint32_t tx = b % R.gx;
    ri = __builtin_amdgcn_readfirstlane((b / R.gx) * blockDim.y + threadIdx.y);
    x = (int)(tx * blockDim.x + threadIdx.x);
    return ri < R.rows;
}

// inner rows: y in [1, ny - 2], z in [1, nz - 2]
__device__ inline void inner_row(const Geom &g, uint32_t ri, int &y, int &z) {
    const uint32_t w = (uint32_t)g.ny - 2u;
    y = 1 + (int)(ri % w);
    z = 1 + (int)(ri / w);
}

// face rows: every row of the z faces, then the y-face rows of the inner z layers
__device__ inline void face_row(const Geom &g, const RowGrid &R, uint32_t ri, int &y, int &z) {
    const uint32_t nzr = (uint32_t)R.zf * (uint32_t)g.ny;
    if (ri < nzr) {
        y = (int)(ri % (uint32_t)g.ny);
        z = ri < (uint32_t)g.ny ? 0 : g.nz - 1;
    } else {
        const uint32_t k = ri - nzr;
        z = 1 + (int)(k / (uint32_t)R.yf);
        y = (k % (uint32_t)R.yf) == 0 ? 0 : g.ny - 1;
    }
}

// Launch shapes of the inner-row and face-row kernels for blocks of bx x by
// (bx a multiple of 64); inner rows may be none (ny or nz below 3).
struct RowLaunch {
    RowGrid inner, face;
    uint32_t inner_blocks, face_blocks;
};

inline RowLaunch row_launch(const Geom &g, int bx, int by, int remap) {
    RowLaunch L;
    RowGrid R;
    R.gx = (uint32_t)((g.nx + bx - 1) / bx);
    R.zf = g.nz > 1 ? 2 : 1;
    R.yf = g.ny > 1 ? 2 : 1;
    R.remap = remap;
    R.rows = (g.ny > 2 && g.nz > 2) ? (uint32_t)(g.ny - 2) * (uint32_t)(g.nz - 2) : 0u;
    L.inner_blocks = R.gx * ((R.rows + by - 1) / by);
    R.aligned = L.inner_blocks & ~7u;
    L.inner = R;
    R.rows = (uint32_t)R.zf * (uint32_t)g.ny + (g.nz > 2 ? (uint32_t)(g.nz - 2) * (uint32_t)R.yf : 0u);
    L.face_blocks = R.gx * ((R.rows + by - 1) / by);
    R.aligned = L.face_blocks & ~7u;
    R.remap = 0;
    L.face = R;
    return L;
}

}  // namespace clbm

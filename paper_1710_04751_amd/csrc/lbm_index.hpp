// Index arithmetic of the fused step: where each population a cell pulls
// (eq. 2b, 13b) and stores lives in the row-group layout, relative to the
// block's window of the state.  Host and device functions, so the same code
// the kernel runs can be enumerated on the CPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {
namespace idx {

constexpr int EX15[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int EY15[15] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int EZ15[15] = {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
constexpr int OPP15[15] = {0, 2, 1, 4, 3, 6, 5, 14, 13, 12, 11, 10, 9, 8, 7};
constexpr int EX7[7] = {0, 1, -1, 0, 0, 0, 0};
constexpr int EY7[7] = {0, 0, 0, 1, -1, 0, 0};
constexpr int EZ7[7] = {0, 0, 0, 0, 0, 1, -1};
constexpr int OPP7[7] = {0, 2, 1, 4, 3, 6, 5};

// D3Q15 population with the y (fy) and/or z (fz) component of e_a reversed:
// the specular image of a at a y or z face.
__host__ __device__ constexpr int mirror15(int a, bool fy, bool fz) {
    for (int b = 0; b < 15; ++b)
        if (EX15[b] == EX15[a] && EY15[b] == (fy ? -EY15[a] : EY15[a]) &&
            EZ15[b] == (fz ? -EZ15[a] : EZ15[a]))
            return b;
    return -1;
}

// log2 of the rows per population run: the largest power of two R with
// R*nx values of one population within 32 KB, and R no more than the rows.
__host__ __device__ inline int rows_log2(int64_t nx, int64_t ny, int64_t nz, int vbytes) {
    const int64_t row_bytes = nx * vbytes;
    const int64_t nrows = ny * nz;
    int gs = 0;
    while ((row_bytes << (gs + 1)) <= 32768 && ((int64_t)2 << gs) <= nrows) ++gs;
    return gs;
}

// The window of the state one block of the step addresses: from the group
// of row (z-1, y0-1) -- the first row a cell of a tile starting at row
// (z, y0) can pull from, clamped at row 0 -- to the end of the state, in
// values (elements) from base = group g0.  rq = 15 + q runs per group.
struct Window {
    uint32_t nx, ny, gs, gmask;
    uint32_t run;    // values per population run (one group of rows)
    uint32_t glen;   // values per group
    uint32_t g0;     // first group of the window
    uint32_t bytes;  // window length in bytes, clamped to 2^32 - 1
};

__host__ __device__ inline Window window_of(int z, int y0, int nx, int ny, int nz, int gs,
                                            int rq, int vbytes) {
    Window w;
    w.nx = (uint32_t)nx;
    w.ny = (uint32_t)ny;
    w.gs = (uint32_t)gs;
    w.gmask = (1u << gs) - 1u;
    w.run = w.nx << gs;
    w.glen = (uint32_t)rq * w.run;
    const uint32_t r0 = (uint32_t)z * w.ny + (uint32_t)y0;
    w.g0 = (r0 > w.ny ? r0 - w.ny - 1 : 0u) >> gs;
    const uint32_t ngroups = (w.ny * (uint32_t)nz + w.gmask) >> gs;
    const uint64_t b = (uint64_t)(ngroups - w.g0) * w.glen * (uint64_t)vbytes;
    w.bytes = b > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)b;
    return w;
}

// Offset of row r's first value in population run 0, from the window base.
__host__ __device__ inline uint32_t row_at(const Window& w, uint32_t r) {
    return ((r >> w.gs) - w.g0) * w.glen + (r & w.gmask) * w.nx;
}

// Wall flags of one cell.
struct CellAt {
    int x, y, z;
    bool xlo, xhi, ylo, yhi, zlo, zhi;
    uint32_t r;    // row z*ny + y
    uint32_t own;  // offset of the cell in population run 0
};

__host__ __device__ inline CellAt cell_at(const Window& w, int x, int y, int z, int nx, int ny,
                                          int nz) {
    CellAt c;
    c.x = x;
    c.y = y;
    c.z = z;
    c.xlo = x == 0;
    c.xhi = x == nx - 1;
    c.ylo = y == 0;
    c.yhi = y == ny - 1;
    c.zlo = z == 0;
    c.zhi = z == nz - 1;
    c.r = (uint32_t)z * w.ny + (uint32_t)y;
    c.own = row_at(w, c.r) + (uint32_t)x;
    return c;
}

// Flow population a: pull from x - e_a, or, across any wall, the opposite
// population of the cell itself (half-way bounce-back).  Offset from the
// window base.
__host__ __device__ inline uint32_t flow_load(const Window& w, const CellAt& c, int a) {
    const int ex = EX15[a], ey = EY15[a], ez = EZ15[a];
    const bool o = (ex > 0 && c.xlo) || (ex < 0 && c.xhi) || (ey > 0 && c.ylo) ||
                   (ey < 0 && c.yhi) || (ez > 0 && c.zlo) || (ez < 0 && c.zhi);
    const uint32_t src = row_at(w, c.r - (uint32_t)(ey + ez * (int32_t)w.ny)) + (uint32_t)(c.x - ex);
    return o ? c.own + (uint32_t)OPP15[a] * w.run : src + (uint32_t)a * w.run;
}

// Scalar population a (lattice QT): the offset to load and whether the link
// crosses a Dirichlet wall (then the loaded value enters anti-bounce-back).
// A link whose source lies beyond a Dirichlet wall loads the opposite
// population of the cell (that rule wins on edges); one whose source lies
// beyond adiabatic faces only loads the opposite population (bounce-back)
// or, with SPEC on D3Q15, the population with the crossed components of e_a
// reversed from the cell (x - e_ax, y', z'), y' = y across a y face and
// y - e_ay otherwise, likewise z' (specular reflection).
struct ScalarLoad {
    uint32_t off;
    bool dirichlet;
};

template <int QT, bool SPEC>
__host__ __device__ inline ScalarLoad scalar_load(const Window& w, const CellAt& c, int a) {
    const int ex = QT == 7 ? EX7[a] : EX15[a];
    const int ey = QT == 7 ? EY7[a] : EY15[a];
    const int ez = QT == 7 ? EZ7[a] : EZ15[a];
    const int ob = QT == 7 ? OPP7[a] : OPP15[a];
    const bool outx = (ex > 0 && c.xlo) || (ex < 0 && c.xhi);
    const bool outy = (ey > 0 && c.ylo) || (ey < 0 && c.yhi);
    const bool outz = (ez > 0 && c.zlo) || (ez < 0 && c.zhi);
    const bool o = outx || outy || outz;
    const uint32_t src = row_at(w, c.r - (uint32_t)(ey + ez * (int32_t)w.ny)) + (uint32_t)(c.x - ex);
    uint32_t off = o ? c.own + (uint32_t)(15 + ob) * w.run : src + (uint32_t)(15 + a) * w.run;
    if constexpr (SPEC && QT == 15) {
        if (ey != 0 || ez != 0) {
            const int dy = outy ? 0 : ey, dz = outz ? 0 : ez;
            const uint32_t b = (uint32_t)(outy ? (outz ? mirror15(a, true, true)
                                                       : mirror15(a, true, false))
                                               : mirror15(a, false, true));
            const uint32_t img = row_at(w, c.r - (uint32_t)(dy + dz * (int32_t)w.ny)) +
                                 (uint32_t)(c.x - ex);
            if ((outy || outz) && !outx) off = img + (15u + b) * w.run;
        }
    }
    return ScalarLoad{off, outx};
}

// Store of population a (flow a < 15, scalar 15 + a) of the cell.
__host__ __device__ inline uint32_t store_at(const Window& w, const CellAt& c, int run_index) {
    return c.own + (uint32_t)run_index * w.run;
}

}  // namespace idx
}  // namespace lbm

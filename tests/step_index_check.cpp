// CPU check of the fused step's index arithmetic (paper_1710_04751_amd/csrc/
// lbm_index.hpp, the functions the step kernel runs): for every block a
// launch of a box forms, every load and store offset a checked cell takes
// must (1) lie inside the block's window of the state and (2) address the
// population and cell the pull-streaming and wall rules name, located by the
// documented row-group layout formula written out here independently.
//
// Usage: step_index_check nx ny nz qt value_bytes by spec mode
//   mode 0: every cell of every block (small boxes)
//   mode 1: for every block, the cells x in {0, 1, nx/2, nx-2, nx-1} of its
//           first and last rows, plus every cell on the box's faces
// Prints "ok <checks>" or the first violation, exit status 1.
#include <cstdio>
#include <cstdlib>
#include <cstdint>

#include "../paper_1710_04751_amd/csrc/lbm_index.hpp"

using namespace lbm::idx;

static int nx, ny, nz, qt, vb, by, spec, gs, rq;
static long long checks = 0;

// element index of run `run_index` (flow a, or 15 + scalar a) of cell
// (x, y, z) in the whole state: the row-group layout of include/lbm.h
static int64_t layout_index(int run_index, int x, int y, int z) {
    const int64_t r = (int64_t)z * ny + y;
    const int64_t R = (int64_t)1 << gs;
    return ((r / R) * rq + run_index) * R * nx + (r % R) * nx + x;
}

static void fail(const char* what, int x, int y, int z, int y0, int a, int64_t got, int64_t want) {
    std::printf("FAIL %s: cell (%d,%d,%d) tile row %d pop %d: offset %lld expected %lld\n", what,
                x, y, z, y0, a, (long long)got, (long long)want);
    std::exit(1);
}

static void check_offset(const Window& w, uint32_t off, int64_t want, const char* what, int x,
                         int y, int z, int y0, int a) {
    ++checks;
    // (1) inside the window
    if ((uint64_t)off * vb + vb > (uint64_t)w.bytes) fail(what, x, y, z, y0, a, off, -1);
    // (2) the intended value
    const int64_t global = (int64_t)w.g0 * w.glen + off;
    if (global != want) fail(what, x, y, z, y0, a, global, want);
}

static bool out_of_box(int x, int y, int z) {
    return x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz;
}

template <int QT, bool SPEC>
static void check_cell(int x, int y, int z, int y0) {
    const Window w = window_of(z, y0, nx, ny, nz, gs, rq, vb);
    const CellAt c = cell_at(w, x, y, z, nx, ny, nz);
    // flow: x - e_a, or the opposite population of the cell (bounce-back)
    for (int a = 0; a < 15; ++a) {
        const int sx = x - EX15[a], sy = y - EY15[a], sz = z - EZ15[a];
        const int64_t want = out_of_box(sx, sy, sz) ? layout_index(OPP15[a], x, y, z)
                                                    : layout_index(a, sx, sy, sz);
        check_offset(w, flow_load(w, c, a), want, "flow load", x, y, z, y0, a);
    }
    const int* ex = QT == 7 ? EX7 : EX15;
    const int* ey = QT == 7 ? EY7 : EY15;
    const int* ez = QT == 7 ? EZ7 : EZ15;
    const int* op = QT == 7 ? OPP7 : OPP15;
    for (int a = 0; a < QT; ++a) {
        const int sx = x - ex[a], sy = y - ey[a], sz = z - ez[a];
        const bool outx = sx < 0 || sx >= nx;
        const bool outy = sy < 0 || sy >= ny, outz = sz < 0 || sz >= nz;
        int64_t want;
        if (!outx && !outy && !outz) {
            want = layout_index(15 + a, sx, sy, sz);
        } else if (outx || !SPEC || QT == 7) {
            want = layout_index(15 + op[a], x, y, z);
        } else {
            // specular image: crossed components reversed, from (sx, y', z')
            int b = -1;
            for (int k = 0; k < QT; ++k)
                if (ex[k] == ex[a] && ey[k] == (outy ? -ey[a] : ey[a]) &&
                    ez[k] == (outz ? -ez[a] : ez[a]))
                    b = k;
            want = layout_index(15 + b, sx, outy ? y : sy, outz ? z : sz);
        }
        const ScalarLoad l = scalar_load<QT, SPEC>(w, c, a);
        if (l.dirichlet != outx) fail("dirichlet flag", x, y, z, y0, a, l.dirichlet, outx);
        check_offset(w, l.off, want, "scalar load", x, y, z, y0, a);
    }
    for (int a = 0; a < 15 + QT; ++a)
        check_offset(w, store_at(w, c, a), layout_index(a, x, y, z), "store", x, y, z, y0, a);
}

template <int QT, bool SPEC>
static void run(int mode) {
    const int xs[5] = {0, 1, nx / 2, nx - 2, nx - 1};
    for (int z = 0; z < nz; ++z)
        for (int y0 = 0; y0 < ny; y0 += by) {
            const int y1 = y0 + by - 1 < ny - 1 ? y0 + by - 1 : ny - 1;
            for (int y = y0; y <= y1; ++y) {
                const bool face_row = y == 0 || y == ny - 1 || z == 0 || z == nz - 1;
                if (mode == 0 || face_row) {
                    for (int x = 0; x < nx; ++x) check_cell<QT, SPEC>(x, y, z, y0);
                } else if (y == y0 || y == y1) {
                    for (int x : xs) check_cell<QT, SPEC>(x, y, z, y0);
                } else {
                    check_cell<QT, SPEC>(0, y, z, y0);
                    check_cell<QT, SPEC>(nx - 1, y, z, y0);
                }
            }
        }
}

int main(int argc, char** argv) {
    if (argc != 9) {
        std::printf("usage: %s nx ny nz qt value_bytes by spec mode\n", argv[0]);
        return 2;
    }
    nx = std::atoi(argv[1]);
    ny = std::atoi(argv[2]);
    nz = std::atoi(argv[3]);
    qt = std::atoi(argv[4]);
    vb = std::atoi(argv[5]);
    by = std::atoi(argv[6]);
    spec = std::atoi(argv[7]);
    const int mode = std::atoi(argv[8]);
    gs = rows_log2(nx, ny, nz, vb);
    rq = 15 + qt;
    if (qt == 7)
        spec ? run<7, true>(mode) : run<7, false>(mode);
    else
        spec ? run<15, true>(mode) : run<15, false>(mode);
    std::printf("ok %lld gs %d\n", checks, gs);
    return 0;
}

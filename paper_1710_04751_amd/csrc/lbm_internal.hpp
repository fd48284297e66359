// Host-side declarations shared by the C ABI (lbm_api.cpp) and the kernel
// launchers (lbm_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Geometry of one cavity and the tiling of its step launch.
struct Geom {
    int32_t nx, ny, nz;
    int32_t bx, by;           // threads per block along x, y
    int32_t tiles_x, tiles_y; // blocks per row / per plane
    int32_t gs;               // log2 of the rows per population run (PopLay)
};

// Lattice-unit coefficients, in double; launchers convert to the arithmetic
// type of the kernel.
struct Coefs {
    double omega, omega_bulk, omega_hi;  // flow
    double omega_T, omega_hiT, cs2;      // scalar
    double gbeta, T_ref, T_hot, T_cold;
    double src;                          // uniform scalar source R
    double alpha;                        // for the Nusselt number
    int32_t fourth_maxwell;
    int32_t sr;                          // FP16 storage: stochastic rounding
    uint32_t seed;                       // step index, the random stream's key
    int32_t spec;                        // scalar adiabatic faces: specular reflection
};

// Layout of one stored state (A or B), row groups interleaved.  The x-rows
// r = z*ny + y are taken in groups of R = 2^gs consecutive rows; a group is
// stored as rq = 15 + q runs of R*nx values, one run per population (flow
// 0..14, then scalar 0..q-1), each run holding its R rows one after another,
// x fastest.  Flow population a of cell (x, y, z) sits at
// F[((r >> gs)*rq + a)*R*nx + (r & (R-1))*nx + x]; G points 15 runs past F,
// so scalar population a sits at the same position from G.  The state is
// padded to a whole number of groups.
struct PopLay {
    int32_t nx;  // values per row
    int32_t rq;  // runs per group: 15 + q
    int32_t gs;  // log2 of the rows per group
};

// One stored state: base of the flow runs and of the scalar runs.
struct StateBuf {
    void* F;
    void* G;
};

enum class Prec : int32_t { FP64 = 0, FP32 = 1, FP32_S16 = 2 };

int value_bytes(Prec p);

hipError_t launch_step(Prec p, int qt, bool general, const Geom& g, StateBuf in,
                       StateBuf out, const Coefs& c, hipStream_t s);
hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t s);
// Rest state: zero-fills state_bytes at state (both buffers), then, with a
// scalar source, writes the scalar equilibrium at T = -R/2 into st.
hipError_t launch_init_rest(Prec p, int qt, const Geom& g, PopLay pl, void* state,
                            size_t state_bytes, StateBuf st, const Coefs& c, hipStream_t s);
// stag: device scratch of 4 doubles (16-byte aligned) for the staggered sums
hipError_t launch_init_macros(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st,
                              const float* ux, const float* uy, const float* uz, const float* T,
                              double* stag, const Coefs& c, hipStream_t s);
hipError_t launch_macros(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st, void* rho,
                         void* ux, void* uy, void* uz, void* T, bool fp64, const Coefs& c,
                         hipStream_t s);
hipError_t launch_nusselt(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st,
                          double* local_hot, double* local_cold, double* result,
                          const Coefs& c, hipStream_t s);
hipError_t launch_centerlines(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st,
                              double* u_line, double* w_line, const Coefs& c, double u0,
                              hipStream_t s);
hipError_t launch_symmetrize(const Geom& g, float* ux, float* uy, float* uz, float* T, double T0,
                             hipStream_t s);
hipError_t launch_residual(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st, void* snapshot,
                           bool compare, unsigned long long* max_bits, unsigned int* bad_flag,
                           hipStream_t s);
hipError_t launch_get_pops(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st, double* F,
                           double* G, hipStream_t s);
hipError_t launch_set_pops(Prec p, int qt, const Geom& g, PopLay pl, StateBuf st,
                           const double* F, const double* G, hipStream_t s);
hipError_t launch_gather_cells(Prec p, int qt, int64_t ncell, PopLay pl, StateBuf st,
                               const int64_t* cells, int64_t n, double* F, double* G,
                               hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
const char* step_kernel_name(Prec p, int qt, bool general);

}  // namespace lbm

// Host-side state of a solver handle and the helpers the C ABI and the
// batched driver share.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

namespace lbm {

struct Layout {
    int64_t ncell;
    PopLay pl;            // row groups interleaved: (15 + q) runs per group of rows
    size_t state_bytes;   // one of A, B
    size_t off_A, off_B, off_snap, off_nu, off_red, total;
};

lbm_status fail(lbm_status s, const std::string& msg);
lbm_status hip_fail(hipError_t e, const char* what);
bool validate(const lbm_params* p, lbm_lattice* L, std::string* why);
// Whether the general collision kernels run: higher-order rates other than
// 1, or a scalar source.
inline bool uses_general_path(const lbm_params* p) {
    return p->omega_hi != 1.0 || p->omega_hi_T != 1.0 || p->R != 0.0;
}
Layout layout_of(const lbm_params* p);
// log2 of the rows per population run: the largest power of two R with
// R*nx values of one population within 32 KB, and R no more than the rows.
int run_rows_log2(const lbm_params* p);
void default_block(int nx, int* bx, int* by);
// Create a handle over caller memory without touching the device.
lbm_status make_handle(const lbm_params* p, void* workspace, size_t bytes, void* stream,
                       lbm_handle** out);
// Wall Nusselt numbers of h's current state with the local profiles in
// prof_hot / prof_cold (ny*nz doubles each) and the eight reduced values in
// result (device memory); copies the profiles to local_hot / local_cold when
// given, then synchronises and fills out.
lbm_status nusselt_into(lbm_handle* h, double* prof_hot, double* prof_cold, double* result,
                        lbm_nu* out, double* local_hot, double* local_cold);

}  // namespace lbm

struct lbm_handle {
    lbm_params p;
    lbm_lattice L;
    lbm::Coefs c;
    lbm::Layout lay;
    char* ws;
    hipStream_t stream;
    int cur;  // 0: state in A, 1: state in B
    int64_t steps;
    bool snap_valid;
    bool general;
    lbm::Geom geom;
    lbm_batch* owner;  // set for members of a batch (the batch steps them)
    int device;        // HIP device current at creation (-1 if unknown)

    lbm::StateBuf buf(int which) const {
        char* base = ws + (which ? lay.off_B : lay.off_A);
        const int vb = lbm::value_bytes((lbm::Prec)p.precision);
        return lbm::StateBuf{base, base + ((size_t)15 * lay.pl.nx * vb << lay.pl.gs)};
    }
    double* nu_hot() const { return (double*)(ws + lay.off_nu); }
    double* nu_cold() const { return nu_hot() + (size_t)p.ny * p.nz; }
    double* red() const { return (double*)(ws + lay.off_red); }
};

namespace lbm {
// Stopping rule of a run to steady state, fed one residual per check.
struct SteadyTracker {
    double best = INFINITY;
    int64_t best_step = -1;
    int32_t since = 0;  // checks since the last new minimum
    // Returns an lbm_steady value once the run should stop, else -1.
    int update(double res, int64_t step, double tol, int32_t plateau_checks, double floor,
               int32_t stall_checks) {
        if (!std::isfinite(res)) return res != res ? LBM_STEADY_UNSTABLE : -1;
        if (res < tol) {
            best_step = step;
            return LBM_STEADY_TOL;
        }
        if (res < best) {
            best = res;
            best_step = step;
            since = 0;
            return -1;
        }
        ++since;
        if (plateau_checks > 0 && since >= plateau_checks && best < floor)
            return LBM_STEADY_PLATEAU;
        if (stall_checks > 0 && since >= stall_checks && !(best < floor))
            return LBM_STEADY_STALLED;
        return -1;
    }
};

void set_geom(lbm_handle* h, int bx, int by);
// A member of a batch may be re-initialised only at an even batch step.
bool batch_allows_reinit(const lbm_batch* b);
}

// C ABI of the cascaded double-distribution LBM library (see include/lbm.h).
#include "../../include/lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_handle.hpp"
#include "lbm_index.hpp"

using namespace lbm;

thread_local std::string g_err;

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
}  // namespace

namespace lbm {


lbm_status fail(lbm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

lbm_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_ERR_HIP;
}



// Lattice values from parameters (reading of Sec. 3: the buoyancy velocity
// scale sqrt(g beta dT L) is u0, L = nx; Ra = g beta dT L^3/(nu alpha),
// Pr = nu/alpha; nu = (1/omega - 1/2)/3 (Appendix A), alpha = cs2 (1/omega_T
// - 1/2) (eq. 23)).
bool derive(const lbm_params* p, lbm_lattice* L, std::string* why) {
    const double dT = p->T_hot - p->T_cold;
    if (p->lattice_units) {
        L->nu = p->nu;
        L->alpha = p->alpha;
        L->gbeta = p->gbeta;
    } else {
        if (!(p->Ra > 0) || !(p->Pr > 0) || !(p->u0 > 0)) {
            *why = "Ra, Pr and u0 must be positive";
            return false;
        }
        if (!(dT > 0)) {
            *why = "T_hot must exceed T_cold";
            return false;
        }
        const double Lx = (double)p->nx;
        L->gbeta = p->u0 * p->u0 / (dT * Lx);
        L->nu = p->u0 * Lx * std::sqrt(p->Pr / p->Ra);
        L->alpha = L->nu / p->Pr;
    }
    if (!(L->nu > 0) || !(L->alpha > 0) || !std::isfinite(L->gbeta)) {
        *why = "nu and alpha must be positive";
        return false;
    }
    L->omega_nu = 1.0 / (3.0 * L->nu + 0.5);
    L->omega_bulk = p->omega_bulk > 0 ? p->omega_bulk : L->omega_nu;
    L->omega_T = 1.0 / (L->alpha / p->cs2_T + 0.5);
    L->T_ref = 0.5 * (p->T_hot + p->T_cold);
    return true;
}

bool validate(const lbm_params* p, lbm_lattice* L, std::string* why) {
    if (!p) {
        *why = "null parameters";
        return false;
    }
    if (p->nx < 4 || p->ny < 4 || p->nz < 4) {
        *why = "each of nx, ny, nz must be >= 4";
        return false;
    }
    if (p->thermal_q != 7 && p->thermal_q != 15) {
        *why = "thermal_q must be 7 or 15";
        return false;
    }
    if (p->precision < 0 || p->precision > 2) {
        *why = "unknown precision";
        return false;
    }
    if (p->round_stochastic != 0 && (p->round_stochastic != 1 || p->precision != LBM_FP32_S16)) {
        *why = "round_stochastic is 0, or 1 with FP16 storage";
        return false;
    }
    if (p->scalar_specular != 0 && p->scalar_specular != 1) {
        *why = "scalar_specular is 0 or 1";
        return false;
    }
    if (!std::isfinite(p->R)) {
        *why = "the scalar source R must be finite";
        return false;
    }
    if (!(p->cs2_T > 0) || !(p->cs2_T < 1.0 / 3.0 + 1e-12)) {
        *why = "cs2_T must lie in (0, 1/3]";
        return false;
    }
    if (!p->lattice_units && p->u0 / std::sqrt(1.0 / 3.0) > 0.3) {
        *why = "u0 / c_s exceeds 0.3";
        return false;
    }
    if (!derive(p, L, why)) return false;
    auto ok = [](double w) { return w > 0 && w < 2; };
    if (!ok(L->omega_nu) || !ok(L->omega_T) || !ok(L->omega_bulk) || !ok(p->omega_hi) ||
        !ok(p->omega_hi_T)) {
        *why = "a relaxation rate lies outside (0, 2)";
        return false;
    }
    const int bx = p->block_x, by = p->block_y;
    if (bx || by) {
        if (bx <= 0 || by <= 0 || (bx * by) % 64 || bx * by > 1024) {
            *why = "block_x * block_y must be a positive multiple of 64, at most 1024";
            return false;
        }
    }
    const int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
    const int vb = value_bytes((Prec)p->precision);
    // The step kernel addresses a window of at most 3 ny + 2 rows (the rows
    // of a tile and one plane plus one row on either side) widened to whole
    // row groups, with 32-bit byte offsets; cell indices are 32-bit.
    const int64_t grp = (int64_t)1 << run_rows_log2(p);
    const uint64_t window = (uint64_t)(3 * (int64_t)p->ny + 2 + 2 * grp) * (15 + p->thermal_q) *
                            (uint64_t)p->nx * (uint64_t)vb;
    if (window >= (1ull << 32) || ncell >= (1ll << 31)) {
        *why = "grid too large for 32-bit cell indices and step-window offsets";
        return false;
    }
    return true;
}

int run_rows_log2(const lbm_params* p) {
    return idx::rows_log2(p->nx, p->ny, p->nz, value_bytes((Prec)p->precision));
}

Layout layout_of(const lbm_params* p) {
    Layout l;
    l.ncell = (int64_t)p->nx * p->ny * p->nz;
    l.pl.nx = p->nx;
    l.pl.rq = 15 + p->thermal_q;
    l.pl.gs = run_rows_log2(p);
    const int vb = value_bytes((Prec)p->precision);
    // whole row groups: the last one is padded when the rows do not fill it
    const int64_t grp = (int64_t)1 << l.pl.gs;
    const int64_t rows = ((int64_t)p->ny * p->nz + grp - 1) / grp * grp;
    l.state_bytes = align_up((size_t)(15 + p->thermal_q) * (size_t)rows * p->nx * vb, kAlign);
    l.off_A = 0;
    l.off_B = l.state_bytes;
    l.off_snap = 2 * l.state_bytes;
    const size_t snap_bytes = align_up((size_t)l.ncell * (p->precision == LBM_FP64 ? 8 : 4), kAlign);
    l.off_nu = l.off_snap + snap_bytes;
    // Nusselt profiles (2 ny nz) or centreline profiles (nx + nz) share it
    const size_t nu_vals = std::max((size_t)2 * p->ny * p->nz, (size_t)p->nx + p->nz);
    const size_t nu_bytes = align_up(nu_vals * sizeof(double), kAlign);
    l.off_red = l.off_nu + nu_bytes;
    l.total = l.off_red + kAlign;
    return l;
}

// Fastest measured shape for large boxes is 128 x 2 (256 threads); small
// boxes use rows rounded up to 16 cells.
void default_block(int nx, int* bx, int* by) {
    int b = nx <= 16 ? 16 : nx <= 32 ? 32 : nx <= 64 ? 64 : 128;
    *bx = b;
    *by = std::max(1, 256 / b);
}


void set_geom(lbm_handle* h, int bx, int by) {
    h->geom.nx = h->p.nx;
    h->geom.ny = h->p.ny;
    h->geom.nz = h->p.nz;
    h->geom.bx = bx;
    h->geom.by = by;
    h->geom.tiles_x = (h->p.nx + bx - 1) / bx;
    h->geom.tiles_y = (h->p.ny + by - 1) / by;
    h->geom.gs = h->lay.pl.gs;
}

lbm_status make_handle(const lbm_params* p, void* workspace, size_t bytes, void* stream,
                       lbm_handle** out) {
    std::string why;
    lbm_lattice L;
    if (!out) return fail(LBM_ERR_ARG, "null output handle");
    *out = nullptr;
    if (!validate(p, &L, &why)) return fail(LBM_ERR_ARG, why);
    const Layout lay = layout_of(p);
    if (!workspace || bytes < lay.total)
        return fail(LBM_ERR_ARG, "workspace missing or smaller than lbm_workspace_bytes()");
    if (((uintptr_t)workspace) % kAlign)
        return fail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) return fail(LBM_ERR_STATE, "out of host memory");
    h->p = *p;
    h->L = L;
    h->lay = lay;
    h->ws = (char*)workspace;
    h->stream = (hipStream_t)stream;
    h->cur = 0;
    h->steps = 0;
    h->snap_valid = false;
    h->general = uses_general_path(p);
    h->c.omega = L.omega_nu;
    h->c.omega_bulk = L.omega_bulk;
    h->c.omega_hi = p->omega_hi;
    h->c.omega_T = L.omega_T;
    h->c.omega_hiT = p->omega_hi_T;
    h->c.cs2 = p->cs2_T;
    h->c.gbeta = L.gbeta;
    h->c.T_ref = L.T_ref;
    h->c.T_hot = p->T_hot;
    h->c.T_cold = p->T_cold;
    h->c.src = p->R;
    h->c.alpha = L.alpha;
    h->c.fourth_maxwell = p->fourth_maxwell;
    h->c.sr = p->round_stochastic;
    h->c.seed = 0;
    h->c.spec = p->scalar_specular;
    int bx = p->block_x, by = p->block_y;
    if (!bx || !by) default_block(p->nx, &bx, &by);
    set_geom(h, bx, by);
    h->owner = nullptr;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
    *out = h;
    return LBM_OK;
}

lbm_status nusselt_into(lbm_handle* h, double* prof_hot, double* prof_cold, double* result,
                        lbm_nu* out, double* local_hot, double* local_cold) {
    hipError_t e = launch_nusselt((Prec)h->p.precision, h->p.thermal_q, h->geom, h->lay.pl,
                                  h->buf(h->cur), prof_hot, prof_cold, result, h->c, h->stream);
    if (e != hipSuccess) return hip_fail(e, "nusselt");
    const size_t nb = (size_t)h->p.ny * h->p.nz * sizeof(double);
    if (local_hot) {
        e = hipMemcpyAsync(local_hot, prof_hot, nb, hipMemcpyDeviceToDevice, h->stream);
        if (e != hipSuccess) return hip_fail(e, "nusselt copy");
    }
    if (local_cold) {
        e = hipMemcpyAsync(local_cold, prof_cold, nb, hipMemcpyDeviceToDevice, h->stream);
        if (e != hipSuccess) return hip_fail(e, "nusselt copy");
    }
    double r[8];
    e = hipMemcpyAsync(r, result, sizeof r, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "nusselt copy");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "nusselt sync");
    out->nu_hot_wall = r[0];
    out->nu_cold_wall = r[1];
    out->nu_hot_mid = r[2];
    out->nu_cold_mid = r[3];
    out->nu_max = r[4];
    out->z_max = r[5];
    out->nu_min = r[6];
    out->z_min = r[7];
    for (double v : r)
        if (!std::isfinite(v)) return fail(LBM_ERR_UNSTABLE, "non-finite Nusselt number");
    return LBM_OK;
}

}  // namespace lbm

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_params_init(lbm_params* p, int32_t n, double Ra) {
    if (!p) return fail(LBM_ERR_ARG, "null parameters");
    std::memset(p, 0, sizeof *p);
    p->nx = p->ny = p->nz = n;
    p->thermal_q = 7;
    p->precision = LBM_FP32;
    p->fourth_maxwell = 0;
    p->Ra = Ra;
    p->Pr = 0.71;
    p->u0 = 0.05;
    p->T_hot = 0.5;
    p->T_cold = -0.5;
    p->cs2_T = 1.0 / 3.0;
    p->omega_bulk = 0.0;
    p->omega_hi = 1.0;
    p->omega_hi_T = 1.0;
    p->R = 0.0;
    return LBM_OK;
}

lbm_status lbm_params_lattice(const lbm_params* p, lbm_lattice* out) {
    std::string why;
    lbm_lattice L;
    if (!out) return fail(LBM_ERR_ARG, "null output");
    if (!validate(p, &L, &why)) return fail(LBM_ERR_ARG, why);
    *out = L;
    return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_params* p) {
    std::string why;
    lbm_lattice L;
    if (!validate(p, &L, &why)) {
        g_err = why;
        return 0;
    }
    return layout_of(p).total;
}

lbm_status lbm_create(const lbm_params* p, void* workspace, size_t bytes, void* stream,
                      lbm_handle** out) {
    lbm_handle* h = nullptr;
    lbm_status s = make_handle(p, workspace, bytes, stream, &h);
    if (s != LBM_OK) {
        if (out) *out = nullptr;
        return s;
    }
    s = lbm_init_rest(h);
    if (s != LBM_OK) {
        delete h;
        *out = nullptr;
        return s;
    }
    *out = h;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_handle* h) {
    if (h && h->owner) return fail(LBM_ERR_STATE, "a batch member is released with its batch");
    delete h;
    return LBM_OK;
}

lbm_status lbm_get_lattice(const lbm_handle* h, lbm_lattice* out) {
    if (!h || !out) return fail(LBM_ERR_ARG, "null argument");
    *out = h->L;
    return LBM_OK;
}

int64_t lbm_steps_done(const lbm_handle* h) { return h ? h->steps : -1; }

lbm_status lbm_init_rest(lbm_handle* h) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->owner && !batch_allows_reinit(h->owner))
        return fail(LBM_ERR_STATE, "batch member re-initialised at an odd batch step");
    hipError_t e = launch_init_rest((Prec)h->p.precision, h->p.thermal_q, h->geom, h->lay.pl,
                                    h->ws + h->lay.off_A, h->lay.state_bytes, h->buf(0), h->c,
                                    h->stream);
    if (e != hipSuccess) return hip_fail(e, "init_rest");
    h->cur = 0;
    h->steps = 0;
    h->snap_valid = false;
    return LBM_OK;
}

lbm_status lbm_init_macros(lbm_handle* h, const float* ux, const float* uy, const float* uz,
                           const float* T) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->owner && !batch_allows_reinit(h->owner))
        return fail(LBM_ERR_STATE, "batch member re-initialised at an odd batch step");
    // red()[10..13]: scratch of the staggered momentum sums
    hipError_t e = launch_init_macros((Prec)h->p.precision, h->p.thermal_q, h->geom, h->lay.pl,
                                      h->buf(0), ux, uy, uz, T, h->red() + 10, h->c, h->stream);
    if (e != hipSuccess) return hip_fail(e, "init_macros");
    h->cur = 0;
    h->steps = 0;
    h->snap_valid = false;
    return LBM_OK;
}

lbm_status lbm_step(lbm_handle* h, int64_t nsteps) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->owner) return fail(LBM_ERR_STATE, "batch members are stepped by lbm_batch_step");
    if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
    const Prec pr = (Prec)h->p.precision;
    for (int64_t i = 0; i < nsteps; ++i) {
        h->c.seed = (uint32_t)h->steps;
        hipError_t e = launch_step(pr, h->p.thermal_q, h->general, h->geom,
                                   h->buf(h->cur), h->buf(1 - h->cur), h->c, h->stream);
        if (e != hipSuccess) return hip_fail(e, "step");
        h->cur = 1 - h->cur;
        ++h->steps;
    }
    return LBM_OK;
}

lbm_status lbm_macros(lbm_handle* h, void* rho, void* ux, void* uy, void* uz, void* T, int fp64) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    hipError_t e = launch_macros((Prec)h->p.precision, h->p.thermal_q, h->geom, h->lay.pl,
                                 h->buf(h->cur), rho, ux, uy, uz, T, fp64 != 0, h->c, h->stream);
    if (e != hipSuccess) return hip_fail(e, "macros");
    return LBM_OK;
}

lbm_status lbm_nusselt(lbm_handle* h, lbm_nu* out, double* local_hot, double* local_cold) {
    if (!h || !out) return fail(LBM_ERR_ARG, "null argument");
    return nusselt_into(h, h->nu_hot(), h->nu_cold(), h->red(), out, local_hot, local_cold);
}

lbm_status lbm_residual(lbm_handle* h, double* max_dT) {
    if (!h || !max_dT) return fail(LBM_ERR_ARG, "null argument");
    // red()[8] holds the max bits, red()[9] the flag; cleared by a kernel so
    // that the sequence stays free of memset nodes under stream capture
    unsigned long long* mb = (unsigned long long*)(h->red() + 8);
    unsigned int* bad = (unsigned int*)(h->red() + 9);
    hipError_t e = launch_fill_zero(mb, 16, h->stream);
    if (e != hipSuccess) return hip_fail(e, "residual clear");
    e = launch_residual((Prec)h->p.precision, h->p.thermal_q, h->geom, h->lay.pl, h->buf(h->cur),
                        h->ws + h->lay.off_snap, h->snap_valid, mb, bad, h->stream);
    if (e != hipSuccess) return hip_fail(e, "residual");
    unsigned long long r[2];
    e = hipMemcpyAsync(r, mb, sizeof r, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "residual copy");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "residual sync");
    const bool was_valid = h->snap_valid;
    h->snap_valid = true;
    if ((unsigned int)r[1] != 0) {
        *max_dT = NAN;
        return fail(LBM_ERR_UNSTABLE, "NaN or Inf in the temperature field");
    }
    double m;
    std::memcpy(&m, &r[0], sizeof m);
    *max_dT = was_valid ? m : INFINITY;
    return LBM_OK;
}

namespace {
// Maximum of v[0..n) at positions (i + 1/2)/n, refined by the parabola
// through the largest sample and its neighbours.
void parabola_peak(const double* v, int n, double* vmax, double* pos) {
    int k = 0;
    for (int i = 1; i < n; ++i)
        if (v[i] > v[k]) k = i;
    double off = 0, val = v[k];
    if (k > 0 && k < n - 1) {
        const double a = v[k - 1], b = v[k], c = v[k + 1];
        const double curv = a - 2 * b + c;
        if (curv < 0) {
            off = 0.5 * (a - c) / curv;
            val = b - 0.25 * (a - c) * off;
        }
    }
    *vmax = val;
    *pos = (k + 0.5 + off) / n;
}
}  // namespace

lbm_status lbm_centerlines(lbm_handle* h, double* u_line, double* w_line, lbm_peaks* peaks) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    double* uu = h->nu_hot();  // scratch for the profiles
    double* ww = uu + h->p.nz;
    hipError_t e = launch_centerlines((Prec)h->p.precision, h->p.thermal_q, h->geom, h->lay.pl,
                                      h->buf(h->cur), uu, ww, h->c, h->p.u0, h->stream);
    if (e != hipSuccess) return hip_fail(e, "centerlines");
    if (u_line) {
        e = hipMemcpyAsync(u_line, uu, sizeof(double) * h->p.nz, hipMemcpyDeviceToDevice,
                           h->stream);
        if (e != hipSuccess) return hip_fail(e, "centerlines copy");
    }
    if (w_line) {
        e = hipMemcpyAsync(w_line, ww, sizeof(double) * h->p.nx, hipMemcpyDeviceToDevice,
                           h->stream);
        if (e != hipSuccess) return hip_fail(e, "centerlines copy");
    }
    if (!peaks) return LBM_OK;
    std::vector<double> hv((size_t)h->p.nz + h->p.nx);
    e = hipMemcpyAsync(hv.data(), uu, sizeof(double) * hv.size(), hipMemcpyDeviceToHost,
                       h->stream);
    if (e != hipSuccess) return hip_fail(e, "centerlines copy");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "centerlines sync");
    for (double v : hv)
        if (!std::isfinite(v)) return fail(LBM_ERR_UNSTABLE, "non-finite velocity");
    parabola_peak(hv.data(), h->p.nz, &peaks->u_max, &peaks->u_pos);
    // distance from the cold wall: reverse the x profile
    std::vector<double> wr(hv.rbegin(), hv.rbegin() + h->p.nx);
    parabola_peak(wr.data(), h->p.nx, &peaks->w_max, &peaks->w_pos);
    return LBM_OK;
}

lbm_status lbm_symmetrize(lbm_handle* h, float* ux, float* uy, float* uz, float* T) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    hipError_t e = launch_symmetrize(h->geom, ux, uy, uz, T, h->c.T_ref, h->stream);
    if (e != hipSuccess) return hip_fail(e, "symmetrize");
    return LBM_OK;
}

lbm_status lbm_run_to_steady(lbm_handle* h, double tol, int64_t check_every, int64_t max_steps,
                             int32_t plateau_checks, double plateau_floor, int32_t stall_checks,
                             int64_t* steps, int32_t* how, double* last_residual) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->owner) return fail(LBM_ERR_STATE, "batch members are run by lbm_batch_run_to_steady");
    if (check_every <= 0 || (check_every & 1) || max_steps < 0 || plateau_checks < 0 ||
        stall_checks < 0)
        return fail(LBM_ERR_ARG, "check_every must be positive and even, the check counts >= 0");
    double res = INFINITY;
    lbm_status s = lbm_residual(h, &res);  // snapshot
    SteadyTracker tr;
    int result = LBM_STEADY_MAX_STEPS;
    int64_t done = 0;
    while (s == LBM_OK && done < max_steps) {
        s = lbm_step(h, check_every);
        if (s != LBM_OK) return s;
        done += check_every;
        s = lbm_residual(h, &res);
        if (s != LBM_OK) break;
        const int r = tr.update(res, h->steps, tol, plateau_checks, plateau_floor, stall_checks);
        if (r >= 0) {
            result = r;
            break;
        }
    }
    if (s == LBM_ERR_UNSTABLE) result = LBM_STEADY_UNSTABLE;
    if (steps)
        *steps = (result == LBM_STEADY_TOL || result == LBM_STEADY_PLATEAU) ? tr.best_step : -1;
    if (how) *how = result;
    if (last_residual) *last_residual = res;
    return s;
}

lbm_status lbm_get_populations(lbm_handle* h, double* F, double* G) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    hipError_t e = launch_get_pops((Prec)h->p.precision, h->p.thermal_q, h->geom, h->lay.pl,
                                   h->buf(h->cur), F, G, h->stream);
    if (e != hipSuccess) return hip_fail(e, "get_populations");
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_handle* h, const double* F, const double* G) {
    if (!h || !F || !G) return fail(LBM_ERR_ARG, "null argument");
    if (h->owner && !batch_allows_reinit(h->owner))
        return fail(LBM_ERR_STATE, "batch member re-initialised at an odd batch step");
    hipError_t e = launch_set_pops((Prec)h->p.precision, h->p.thermal_q, h->geom, h->lay.pl,
                                   h->buf(0), F, G, h->stream);
    if (e != hipSuccess) return hip_fail(e, "set_populations");
    h->cur = 0;
    h->steps = 0;
    h->snap_valid = false;
    return LBM_OK;
}

lbm_status lbm_gather_cells(lbm_handle* h, const int64_t* cells, int64_t n, double* F, double* G,
                            int check) {
    if (!h || (n > 0 && !cells) || n < 0) return fail(LBM_ERR_ARG, "bad arguments");
    if (check && n > 0) {
        std::vector<int64_t> hc((size_t)n);
        hipError_t e = hipMemcpyAsync(hc.data(), cells, (size_t)n * sizeof(int64_t),
                                      hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "gather_cells check");
        for (int64_t v : hc)
            if (v < 0 || v >= h->lay.ncell) return fail(LBM_ERR_ARG, "cell index out of range");
    }
    hipError_t e = launch_gather_cells((Prec)h->p.precision, h->p.thermal_q, h->lay.ncell,
                                       h->lay.pl, h->buf(h->cur), cells, n, F, G, h->stream);
    if (e != hipSuccess) return hip_fail(e, "gather_cells");
    return LBM_OK;
}

lbm_status lbm_state_info(const lbm_handle* h, const void** F, const void** G,
                          int64_t* pop_stride, int32_t* vbytes) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    StateBuf b = h->buf(h->cur);
    if (F) *F = b.F;
    if (G) *G = b.G;
    if (pop_stride) *pop_stride = (int64_t)h->lay.pl.nx << h->lay.pl.gs;
    if (vbytes) *vbytes = value_bytes((Prec)h->p.precision);
    return LBM_OK;
}

const char* lbm_step_kernel_name(const lbm_handle* h) {
    if (!h) return "";
    return step_kernel_name((Prec)h->p.precision, h->p.thermal_q, h->general);
}

lbm_status lbm_set_block(lbm_handle* h, int32_t bx, int32_t by) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (bx <= 0 || by <= 0 || (bx * by) % 64 || bx * by > 1024)
        return fail(LBM_ERR_ARG, "block_x * block_y must be a positive multiple of 64, at most 1024");
    set_geom(h, bx, by);
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_handle* h, int32_t steps_per_trial, int32_t* out_bx, int32_t* out_by) {
    if (!h || steps_per_trial <= 0) return fail(LBM_ERR_ARG, "bad arguments");
    static const int cand[][2] = {{64, 1},  {64, 2},  {64, 4},  {128, 1}, {128, 2},
                                  {256, 1}, {256, 2}, {512, 1}, {1024, 1}};
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "autotune events");
    float best = 1e30f;
    int bbx = h->geom.bx, bby = h->geom.by;
    lbm_status s = LBM_OK;
    for (auto& cnd : cand) {
        const int bx = cnd[0], by = cnd[1];
        if (bx > 2 * std::max(64, h->p.nx)) continue;  // mostly idle lanes
        set_geom(h, bx, by);
        s = lbm_step(h, 1);  // warm the instruction cache
        if (s != LBM_OK) break;
        e = hipEventRecord(e0, h->stream);
        if (e == hipSuccess) s = lbm_step(h, steps_per_trial);
        if (e == hipSuccess && s == LBM_OK) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess && s == LBM_OK) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess && s == LBM_OK) e = hipEventElapsedTime(&ms, e0, e1);
        if (s != LBM_OK || e != hipSuccess) break;
        if (ms < best) best = ms, bbx = bx, bby = by;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_geom(h, bbx, bby);
    if (s != LBM_OK) return s;
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (out_bx) *out_bx = bbx;
    if (out_by) *out_by = bby;
    return LBM_OK;
}

lbm_status lbm_copy_probe(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
        return fail(LBM_ERR_ARG, "copy probe needs 16-byte aligned pointers and size");
    hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "copy_probe");
    return LBM_OK;
}

}  // extern "C"

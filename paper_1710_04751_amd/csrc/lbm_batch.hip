// Batched form: many independent cavities advanced by one persistent launch
// per step, replayed from a captured hipGraph.
//
// Work decomposition.  A tile is `rows` whole x-rows of one z-plane of one
// cavity, with rows = threads_per_block / nx (all sizes are covered, a block
// wastes at most nx - 1 lanes).  The device holds the list of tiles of the
// active cavities; each block of the persistent grid walks the list with a
// stride of the grid size and updates its tile's cells with update_cell, the
// same per-cell function the single-cavity kernel uses.  Retiring a cavity
// rewrites the list and its length on the device, so a captured graph stays
// valid.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "lbm_handle.hpp"
#include "lbm_step.hpp"

namespace lbm {
namespace kern {

// Device table entry of one member.
struct DevCav {
    void* F[2];      // state A / B (flow runs; the scalar runs follow 15 runs later)
    void* G[2];
    void* snap;      // temperature snapshot of the residual
    PopLay pl;
    int32_t nx, ny, nz;
    int32_t rows;    // x-rows per tile
    int32_t ytiles;  // tiles per z-plane
    uint32_t magic;  // ceil(2^20 / nx): row = (lane * magic) >> 20 for lane < 1024
    KCoef<double> kd;
    KCoef<float> kf;
};

template <typename R>
__device__ __forceinline__ const KCoef<R>& coef_of(const DevCav& c);
template <>
__device__ __forceinline__ const KCoef<double>& coef_of<double>(const DevCav& c) { return c.kd; }
template <>
__device__ __forceinline__ const KCoef<float>& coef_of<float>(const DevCav& c) { return c.kf; }

// tile descriptor: cavity (8 bits) | z (10 bits) | y-tile (14 bits)
__device__ __forceinline__ void decode_tile(uint32_t d, int& cav, int& z, int& yt) {
    cav = (int)(d >> 24);
    z = (int)((d >> 14) & 1023u);
    yt = (int)(d & 0x3FFFu);
}

// keys[c] + key_off: member c's step index, the key of its stochastic
// rounding (FP16 storage), so a member draws the random bits a single run of
// it draws.  key_off is the step's position within a captured graph (the
// device keys advance once per replay, k_batch_advance).
template <typename R, typename S, int QT, bool HG>
__global__ void __launch_bounds__(1024)
k_batch_step(const DevCav* __restrict__ cavs, const uint32_t* __restrict__ tiles,
             const uint32_t* __restrict__ ntiles_p, int parity,
             const uint32_t* __restrict__ keys, uint32_t key_off) {
    const uint32_t ntiles = *ntiles_p;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int c, z, yt;
        decode_tile(tiles[t], c, z, yt);
        const DevCav& C = cavs[c];
        const int r = (int)((threadIdx.x * C.magic) >> 20);
        const int x = (int)threadIdx.x - r * C.nx;
        const int y = yt * C.rows + r;
        if (r >= C.rows || y >= C.ny) continue;
        uint32_t seed = 0;
        if constexpr (std::is_same<S, _Float16>::value) seed = keys[c] + key_off;
        update_cell<R, S, QT, HG>((const S*)C.F[parity], (S*)C.F[1 - parity], x, y, z,
                                  yt * C.rows, C.nx, C.ny, C.nz, C.pl.gs, coef_of<R>(C), seed);
    }
}

// Advance the step keys of the active members by k (one thread per member).
__global__ void k_batch_advance(uint32_t* __restrict__ keys, const int32_t* __restrict__ active,
                                int n, uint32_t k) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && active[i]) keys[i] += k;
}

// Residual of every active member: max |T - T_snapshot| (T = sum of the
// stored scalar populations) into max_bits[c], NaN/Inf into bad[c]; renews
// the snapshot.  compare[c] = 0 only takes the snapshot.
template <typename S, int QT, typename Snap>
__global__ void __launch_bounds__(1024)
k_batch_residual(const DevCav* __restrict__ cavs, const uint32_t* __restrict__ tiles,
                 const uint32_t* __restrict__ ntiles_p, int parity, const int32_t* compare,
                 unsigned long long* max_bits, unsigned int* bad) {
    __shared__ double s_red[16];
    const uint32_t ntiles = *ntiles_p;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int c, z, yt;
        decode_tile(tiles[t], c, z, yt);
        const DevCav& C = cavs[c];
        const int r = (int)((threadIdx.x * C.magic) >> 20);
        const int x = (int)threadIdx.x - r * C.nx;
        const int y = yt * C.rows + r;
        double dev = 0;
        if (r < C.rows && y < C.ny) {
            const uint32_t cell =
                ((uint32_t)z * (uint32_t)C.ny + (uint32_t)y) * (uint32_t)C.nx + (uint32_t)x;
            const S* G = (const S*)C.G[parity];
            double T = 0;
#pragma unroll
            for (int a = 0; a < QT; ++a) T += Store<S>::template ld<double>(G + pop_at(C.pl, a, cell));
            Snap* snap = (Snap*)C.snap;
            const Snap Ts = (Snap)T;
            if (!isfinite(T)) atomicOr(bad + c, 1u);
            if (compare[c]) dev = fabs((double)Ts - (double)snap[cell]);
            snap[cell] = Ts;
        }
        for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o, 64));
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = dev;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = s_red[0];
            for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, s_red[i]);
            if (m > 0) atomicMax(max_bits + c, (unsigned long long)__double_as_longlong(m));
        }
        __syncthreads();
    }
}

// Rebuild the tile list of the active members (one block).
__global__ void __launch_bounds__(1024)
k_batch_compact(const DevCav* __restrict__ cavs, const int32_t* __restrict__ active, int n,
                uint32_t* __restrict__ tiles, uint32_t* __restrict__ ntiles) {
    __shared__ uint32_t off[257];
    if (threadIdx.x == 0) {
        off[0] = 0;
        for (int c = 0; c < n; ++c)
            off[c + 1] = off[c] + (active[c] ? (uint32_t)(cavs[c].nz * cavs[c].ytiles) : 0u);
        *ntiles = off[n];
    }
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        if (!active[c]) continue;
        const uint32_t yts = (uint32_t)cavs[c].ytiles;
        const uint32_t cnt = (uint32_t)cavs[c].nz * yts;
        for (uint32_t j = threadIdx.x; j < cnt; j += blockDim.x) {
            const uint32_t z = j / yts, yt = j - z * yts;
            tiles[off[c] + j] = ((uint32_t)c << 24) | (z << 14) | yt;
        }
    }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace kern

bool batch_allows_reinit(const lbm_batch* b);

}  // namespace lbm

using namespace lbm;
using namespace lbm::kern;

namespace {

constexpr size_t kAlignB = 256;
size_t alignb(size_t v) { return (v + kAlignB - 1) / kAlignB * kAlignB; }

struct BatchLayout {
    size_t off_table, off_tiles, off_ntiles, off_flags, off_res, off_keys, off_members, total;
    std::vector<size_t> member_off, member_bytes;
    size_t max_tiles;
};

bool batch_layout(const lbm_params* p, int n, BatchLayout* L, std::string* why) {
    if (n < 1 || n > 255) {
        *why = "a batch holds 1 to 255 cavities";
        return false;
    }
    size_t max_tiles = 0;
    L->member_off.resize(n);
    L->member_bytes.resize(n);
    for (int i = 0; i < n; ++i) {
        lbm_lattice lat;
        if (!validate(&p[i], &lat, why)) {
            *why = "member " + std::to_string(i) + ": " + *why;
            return false;
        }
        if (p[i].precision != p[0].precision || p[i].thermal_q != p[0].thermal_q ||
            uses_general_path(&p[i]) != uses_general_path(&p[0])) {
            *why = "batch members must share precision, thermal_q and the collision path "
                   "(higher-order rates other than 1 or a scalar source)";
            return false;
        }
        if (p[i].round_stochastic != p[0].round_stochastic) {
            *why = "batch members must share the storage rounding mode";
            return false;
        }
        if (p[i].nx > 1024 || p[i].nz > 1023 || p[i].ny > 16383) {
            *why = "batch members need nx <= 1024, ny <= 16383, nz <= 1023";
            return false;
        }
        max_tiles += (size_t)p[i].ny * p[i].nz;
    }
    L->max_tiles = max_tiles;
    L->off_table = 0;
    L->off_tiles = alignb(sizeof(DevCav) * n);
    L->off_ntiles = L->off_tiles + alignb(max_tiles * sizeof(uint32_t));
    L->off_flags = L->off_ntiles + kAlignB;                    // active[n], compare[n]
    L->off_res = L->off_flags + alignb(2 * n * sizeof(int32_t));  // max bits[n], bad[n]
    L->off_keys = L->off_res + alignb(2 * n * sizeof(unsigned long long));  // step keys[n]
    L->off_members = L->off_keys + alignb(n * sizeof(uint32_t));
    size_t off = L->off_members;
    for (int i = 0; i < n; ++i) {
        L->member_off[i] = off;
        L->member_bytes[i] = layout_of(&p[i]).total;
        off += alignb(L->member_bytes[i]);
    }
    L->total = off;
    return true;
}

}  // namespace

struct lbm_batch {
    int n;
    std::vector<lbm_handle*> mem;
    std::vector<int32_t> active;
    std::vector<double> last_res;
    std::vector<int32_t> last_status;
    char* ws;
    hipStream_t stream;
    BatchLayout lay;
    Prec prec;
    int qt;
    bool general;
    int64_t gsteps;     // steps taken by the batch (global parity)
    int threads, bpc, graph_steps, cu_count;
    int64_t tiles_all;  // tiles of all members at the current block size
    hipGraphExec_t graph;
    bool graph_ok;
    std::vector<DevCav> table;
    bool sr;                          // stochastic rounding: step keys live on the device
    std::vector<uint32_t> keys_host;  // what d_keys() holds (valid once keys_ok)
    bool keys_ok;

    DevCav* d_table() const { return (DevCav*)(ws + lay.off_table); }
    uint32_t* d_tiles() const { return (uint32_t*)(ws + lay.off_tiles); }
    uint32_t* d_ntiles() const { return (uint32_t*)(ws + lay.off_ntiles); }
    int32_t* d_active() const { return (int32_t*)(ws + lay.off_flags); }
    int32_t* d_compare() const { return d_active() + n; }
    unsigned long long* d_maxbits() const { return (unsigned long long*)(ws + lay.off_res); }
    unsigned int* d_bad() const { return (unsigned int*)(d_maxbits() + n); }
    uint32_t* d_keys() const { return (uint32_t*)(ws + lay.off_keys); }
};

namespace lbm {
bool batch_allows_reinit(const lbm_batch* b) { return (b->gsteps & 1) == 0; }
}  // namespace lbm

namespace {

template <typename R>
void fill_kcoef(const lbm_handle* h, KCoef<R>* k) {
    k->f.omega = (R)h->c.omega;
    k->f.omega_bulk = (R)h->c.omega_bulk;
    k->f.omega_hi = (R)h->c.omega_hi;
    k->f.gbeta = (R)h->c.gbeta;
    k->f.T_ref = (R)h->c.T_ref;
    k->f.fourth_maxwell = h->c.fourth_maxwell;
    k->t.omega_T = (R)h->c.omega_T;
    k->t.omega_hiT = (R)h->c.omega_hiT;
    k->t.cs2 = (R)h->c.cs2;
    k->t.src = (R)h->c.src;
    k->sr = h->c.sr;
    k->seed = 0;  // the step keys are device data (k_batch_step)
    k->spec = h->c.spec;
    k->T_hot = (R)h->c.T_hot;
    k->T_cold = (R)h->c.T_cold;
    const double cs2 = h->c.cs2;
    if (h->p.thermal_q == 7) {
        k->w_face = (R)(cs2 / 2);
        k->w_corner = 0;
    } else {
        k->w_face = (R)((cs2 - cs2 * cs2) / 2);
        k->w_corner = (R)(cs2 * cs2 / 8);
    }
}

// Rebuild the host table for the current launch shape and upload it, then
// rebuild the device tile list.
lbm_status upload_table(lbm_batch* b) {
    b->tiles_all = 0;
    for (int i = 0; i < b->n; ++i) {
        const lbm_handle* h = b->mem[i];
        DevCav& d = b->table[i];
        StateBuf A = h->buf(0), B = h->buf(1);
        d.F[0] = A.F;
        d.G[0] = A.G;
        d.F[1] = B.F;
        d.G[1] = B.G;
        d.snap = h->ws + h->lay.off_snap;
        d.pl = h->lay.pl;
        d.nx = h->p.nx;
        d.ny = h->p.ny;
        d.nz = h->p.nz;
        d.rows = std::max(1, b->threads / h->p.nx);
        d.ytiles = (h->p.ny + d.rows - 1) / d.rows;
        b->tiles_all += (int64_t)d.nz * d.ytiles;
        d.magic = (uint32_t)(((1u << 20) + (uint32_t)h->p.nx - 1) / (uint32_t)h->p.nx);
        // the row index must be exact for every lane of the block
        for (uint32_t lane = 0; lane < (uint32_t)b->threads; ++lane)
            if (((lane * d.magic) >> 20) != lane / (uint32_t)h->p.nx)
                return fail(LBM_ERR_ARG, "row decomposition is not exact for this block size");
        fill_kcoef<double>(h, &d.kd);
        fill_kcoef<float>(h, &d.kf);
    }
    hipError_t e = hipMemcpyAsync(b->d_table(), b->table.data(), sizeof(DevCav) * b->n,
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_active(), b->active.data(), sizeof(int32_t) * b->n,
                           hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    hipLaunchKernelGGL(k_batch_compact, dim3(1), dim3(1024), 0, b->stream, b->d_table(),
                       b->d_active(), b->n, b->d_tiles(), b->d_ntiles());
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch compaction");
    // the host table and flags are pageable: make sure they are consumed
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch table sync");
    return LBM_OK;
}

#define LBM_BATCH_DISPATCH(prec, qt, general, ...)                                     \
    do {                                                                               \
        if (prec == Prec::FP64) {                                                      \
            using R = double; using S = double;                                        \
            if (qt == 7) { constexpr int Q = 7; if (general) { constexpr bool G = true; __VA_ARGS__; } else { constexpr bool G = false; __VA_ARGS__; } } \
            else { constexpr int Q = 15; if (general) { constexpr bool G = true; __VA_ARGS__; } else { constexpr bool G = false; __VA_ARGS__; } } \
        } else if (prec == Prec::FP32) {                                               \
            using R = float; using S = float;                                          \
            if (qt == 7) { constexpr int Q = 7; if (general) { constexpr bool G = true; __VA_ARGS__; } else { constexpr bool G = false; __VA_ARGS__; } } \
            else { constexpr int Q = 15; if (general) { constexpr bool G = true; __VA_ARGS__; } else { constexpr bool G = false; __VA_ARGS__; } } \
        } else {                                                                       \
            using R = float; using S = _Float16;                                       \
            if (qt == 7) { constexpr int Q = 7; if (general) { constexpr bool G = true; __VA_ARGS__; } else { constexpr bool G = false; __VA_ARGS__; } } \
            else { constexpr int Q = 15; if (general) { constexpr bool G = true; __VA_ARGS__; } else { constexpr bool G = false; __VA_ARGS__; } } \
        }                                                                              \
    } while (0)

// Grid of the batched kernels: bpc blocks per compute unit walking the tile
// list, or (bpc = 0) one block per tile of the whole batch; blocks beyond the
// active tiles return at once, so the grid stays valid as members retire.
unsigned batch_grid(const lbm_batch* b) {
    return (unsigned)(b->bpc > 0 ? (int64_t)b->cu_count * b->bpc : std::max<int64_t>(1, b->tiles_all));
}

hipError_t launch_one_step(lbm_batch* b, int parity, uint32_t key_off) {
    const dim3 grid(batch_grid(b)), block((unsigned)b->threads);
    LBM_BATCH_DISPATCH(b->prec, b->qt, b->general, {
        hipLaunchKernelGGL((k_batch_step<R, S, Q, G>), grid, block, 0, b->stream, b->d_table(),
                           b->d_tiles(), b->d_ntiles(), parity, (const uint32_t*)b->d_keys(),
                           key_off);
    });
    return hipGetLastError();
}

hipError_t launch_advance(lbm_batch* b, uint32_t k) {
    hipLaunchKernelGGL(k_batch_advance, dim3((b->n + 255) / 256), dim3(256), 0, b->stream,
                       b->d_keys(), (const int32_t*)b->d_active(), b->n, k);
    return hipGetLastError();
}

// With stochastic rounding, make the device step keys equal the members'
// step counts (members re-initialised since the last upload restart at 0).
lbm_status sync_keys(lbm_batch* b) {
    if (!b->sr) return LBM_OK;
    bool same = b->keys_ok;
    for (int i = 0; i < b->n && same; ++i) same = b->keys_host[i] == (uint32_t)b->mem[i]->steps;
    if (same) return LBM_OK;
    for (int i = 0; i < b->n; ++i) b->keys_host[i] = (uint32_t)b->mem[i]->steps;
    hipError_t e = hipMemcpyAsync(b->d_keys(), b->keys_host.data(), sizeof(uint32_t) * b->n,
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // pageable source
    if (e != hipSuccess) return hip_fail(e, "batch step keys");
    b->keys_ok = true;
    return LBM_OK;
}

void drop_graph(lbm_batch* b) {
    if (b->graph_ok) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph_ok = false;
    }
}

lbm_status capture_graph(lbm_batch* b) {
    drop_graph(b);
    if (b->graph_steps <= 0) return LBM_OK;
    hipGraph_t g;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture begin");
    for (int i = 0; i < b->graph_steps; ++i) {
        e = launch_one_step(b, i & 1, (uint32_t)i);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess && b->sr) e = launch_advance(b, (uint32_t)b->graph_steps);
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) return hip_fail(e, "graph capture launch");
    if (e2 != hipSuccess) return hip_fail(e2, "graph capture end");
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    b->graph_ok = true;
    return LBM_OK;
}

void after_steps(lbm_batch* b, int64_t k) {
    b->gsteps += k;
    for (int i = 0; i < b->n; ++i)
        if (b->active[i]) {
            b->mem[i]->steps += k;
            b->mem[i]->cur = (int)(b->gsteps & 1);
            if (b->sr) b->keys_host[i] += (uint32_t)k;  // as k_batch_advance did on the device
        }
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_params* p, int32_t n) {
    BatchLayout L;
    std::string why;
    if (!p || !batch_layout(p, n, &L, &why)) {
        (void)fail(LBM_ERR_ARG, p ? why : std::string("null parameters"));
        return 0;
    }
    return L.total;
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_OK;
    drop_graph(b);
    for (lbm_handle* h : b->mem) {
        if (h) h->owner = nullptr;
        lbm_destroy(h);
    }
    delete b;
    return LBM_OK;
}

lbm_status lbm_batch_create(const lbm_params* p, int32_t n, void* workspace, size_t bytes,
                            void* stream, lbm_batch** out) {
    if (!out) return fail(LBM_ERR_ARG, "null output");
    *out = nullptr;
    BatchLayout L;
    std::string why;
    if (!p || !batch_layout(p, n, &L, &why)) return fail(LBM_ERR_ARG, why);
    if (!workspace || bytes < L.total)
        return fail(LBM_ERR_ARG, "workspace missing or smaller than lbm_batch_workspace_bytes()");
    if ((uintptr_t)workspace % kAlignB) return fail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_ERR_STATE, "out of host memory");
    b->n = n;
    b->ws = (char*)workspace;
    b->stream = (hipStream_t)stream;
    b->lay = L;
    b->prec = (Prec)p[0].precision;
    b->qt = p[0].thermal_q;
    b->general = uses_general_path(&p[0]);
    b->gsteps = 0;
    b->threads = 256;
    b->bpc = 8;
    b->graph_steps = stream ? 100 : 0;  // the legacy default stream cannot be captured
    b->cu_count = cus;
    b->graph_ok = false;
    b->sr = p[0].round_stochastic != 0;
    b->keys_host.assign(n, 0);
    b->keys_ok = false;
    b->active.assign(n, 1);
    b->last_res.assign(n, INFINITY);
    b->last_status.assign(n, LBM_OK);
    b->table.resize(n);
    b->mem.assign(n, nullptr);
    int maxnx = 0;
    for (int i = 0; i < n; ++i) maxnx = std::max(maxnx, p[i].nx);
    if (maxnx > b->threads) b->threads = (maxnx + 63) / 64 * 64;
    for (int i = 0; i < n; ++i) {
        lbm_handle* h = nullptr;
        lbm_status s = make_handle(&p[i], b->ws + L.member_off[i], L.member_bytes[i], stream, &h);
        if (s != LBM_OK) {
            lbm_batch_destroy(b);
            return s;
        }
        b->mem[i] = h;
        s = lbm_init_rest(h);
        h->owner = b;
        if (s != LBM_OK) {
            lbm_batch_destroy(b);
            return s;
        }
    }
    lbm_status s = upload_table(b);
    if (s == LBM_OK) s = capture_graph(b);
    if (s != LBM_OK) {
        lbm_batch_destroy(b);
        return s;
    }
    *out = b;
    return LBM_OK;
}

lbm_handle* lbm_batch_member(lbm_batch* b, int32_t i) {
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->mem[i];
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
    if (!b) return fail(LBM_ERR_ARG, "null batch");
    if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
    for (int i = 0; i < b->n; ++i)
        if (b->active[i] && b->mem[i]->cur != (int)(b->gsteps & 1))
            return fail(LBM_ERR_STATE, "member " + std::to_string(i) +
                                           " was re-initialised out of step with its batch");
    lbm_status ks = sync_keys(b);
    if (ks != LBM_OK) return ks;
    while (nsteps > 0) {
        if (b->graph_ok && (b->gsteps & 1) == 0 && nsteps >= b->graph_steps) {
            hipError_t e = hipGraphLaunch(b->graph, b->stream);
            if (e != hipSuccess) return hip_fail(e, "graph launch");
            after_steps(b, b->graph_steps);
            nsteps -= b->graph_steps;
        } else {
            hipError_t e = launch_one_step(b, (int)(b->gsteps & 1), 0u);
            if (e == hipSuccess && b->sr) e = launch_advance(b, 1u);
            if (e != hipSuccess) return hip_fail(e, "batch step");
            after_steps(b, 1);
            nsteps -= 1;
        }
    }
    return LBM_OK;
}

lbm_status lbm_batch_residuals(lbm_batch* b, double* max_dT, int32_t* status) {
    if (!b) return fail(LBM_ERR_ARG, "null batch");
    std::vector<int32_t> cmp(b->n);
    for (int i = 0; i < b->n; ++i) cmp[i] = b->mem[i]->snap_valid ? 1 : 0;
    hipError_t e = hipMemcpyAsync(b->d_compare(), cmp.data(), sizeof(int32_t) * b->n,
                                  hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(e, "residual flags");
    hipLaunchKernelGGL(k_zero_u64, dim3((2 * b->n + 255) / 256), dim3(256), 0, b->stream,
                       b->d_maxbits(), 2 * b->n);
    const dim3 grid(batch_grid(b)), block((unsigned)b->threads);
    const int parity = (int)(b->gsteps & 1);
    if (b->prec == Prec::FP64) {
        if (b->qt == 7)
            hipLaunchKernelGGL((k_batch_residual<double, 7, double>), grid, block, 0, b->stream,
                               b->d_table(), b->d_tiles(), b->d_ntiles(), parity, b->d_compare(),
                               b->d_maxbits(), b->d_bad());
        else
            hipLaunchKernelGGL((k_batch_residual<double, 15, double>), grid, block, 0, b->stream,
                               b->d_table(), b->d_tiles(), b->d_ntiles(), parity, b->d_compare(),
                               b->d_maxbits(), b->d_bad());
    } else if (b->prec == Prec::FP32) {
        if (b->qt == 7)
            hipLaunchKernelGGL((k_batch_residual<float, 7, float>), grid, block, 0, b->stream,
                               b->d_table(), b->d_tiles(), b->d_ntiles(), parity, b->d_compare(),
                               b->d_maxbits(), b->d_bad());
        else
            hipLaunchKernelGGL((k_batch_residual<float, 15, float>), grid, block, 0, b->stream,
                               b->d_table(), b->d_tiles(), b->d_ntiles(), parity, b->d_compare(),
                               b->d_maxbits(), b->d_bad());
    } else {
        if (b->qt == 7)
            hipLaunchKernelGGL((k_batch_residual<_Float16, 7, float>), grid, block, 0, b->stream,
                               b->d_table(), b->d_tiles(), b->d_ntiles(), parity, b->d_compare(),
                               b->d_maxbits(), b->d_bad());
        else
            hipLaunchKernelGGL((k_batch_residual<_Float16, 15, float>), grid, block, 0, b->stream,
                               b->d_table(), b->d_tiles(), b->d_ntiles(), parity, b->d_compare(),
                               b->d_maxbits(), b->d_bad());
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch residual");
    std::vector<unsigned long long> r(2 * b->n);
    e = hipMemcpyAsync(r.data(), b->d_maxbits(), sizeof(unsigned long long) * 2 * b->n,
                       hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch residual copy");
    const unsigned int* bad = (const unsigned int*)(r.data() + b->n);
    for (int i = 0; i < b->n; ++i) {
        if (!b->active[i]) continue;
        double m;
        std::memcpy(&m, &r[i], sizeof m);
        const bool was = b->mem[i]->snap_valid;
        b->mem[i]->snap_valid = true;
        if (bad[i]) {
            b->last_res[i] = NAN;
            b->last_status[i] = LBM_ERR_UNSTABLE;
        } else {
            b->last_res[i] = was ? m : INFINITY;
            b->last_status[i] = LBM_OK;
        }
    }
    for (int i = 0; i < b->n; ++i) {
        if (max_dT) max_dT[i] = b->last_res[i];
        if (status) status[i] = b->last_status[i];
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_active(lbm_batch* b, const int32_t* active) {
    if (!b || !active) return fail(LBM_ERR_ARG, "null argument");
    // validate the whole request first, so a refused call leaves the batch as it was
    for (int i = 0; i < b->n; ++i)
        if (active[i] && !b->active[i] && b->mem[i]->cur != (int)(b->gsteps & 1))
            return fail(LBM_ERR_STATE, "member " + std::to_string(i) +
                                           " cannot rejoin at this step parity");
    for (int i = 0; i < b->n; ++i) b->active[i] = active[i] ? 1 : 0;
    return upload_table(b);
}

lbm_status lbm_batch_run_to_steady(lbm_batch* b, double tol, int64_t check_every,
                                   int64_t max_steps, int32_t plateau_checks,
                                   double plateau_floor, int32_t stall_checks, int64_t* steps,
                                   int32_t* how, double* last_residual) {
    if (!b || check_every <= 0 || (check_every & 1) || max_steps < 0 || plateau_checks < 0 ||
        stall_checks < 0)
        return fail(LBM_ERR_ARG, "check_every must be positive and even, the check counts >= 0");
    std::vector<SteadyTracker> tr(b->n);
    std::vector<int32_t> end(b->n, LBM_STEADY_MAX_STEPS);
    std::vector<double> res(b->n);
    std::vector<int32_t> rs(b->n);
    // snapshot at the start
    lbm_status s = lbm_batch_residuals(b, res.data(), rs.data());
    if (s != LBM_OK) return s;
    int64_t done = 0;
    while (done < max_steps) {
        bool any = false;
        for (int i = 0; i < b->n; ++i) any = any || b->active[i];
        if (!any) break;
        s = lbm_batch_step(b, check_every);
        if (s != LBM_OK) return s;
        done += check_every;
        s = lbm_batch_residuals(b, res.data(), rs.data());
        if (s != LBM_OK) return s;
        std::vector<int32_t> act = b->active;
        bool changed = false;
        for (int i = 0; i < b->n; ++i) {
            if (!b->active[i]) continue;
            const int r = rs[i] != LBM_OK
                              ? (int)LBM_STEADY_UNSTABLE
                              : tr[i].update(res[i], b->mem[i]->steps, tol, plateau_checks,
                                             plateau_floor, stall_checks);
            if (r >= 0) {
                end[i] = r;
                act[i] = 0;
                changed = true;
            }
        }
        if (changed) {
            s = lbm_batch_set_active(b, act.data());
            if (s != LBM_OK) return s;
        }
    }
    for (int i = 0; i < b->n; ++i) {
        const bool ok = end[i] == LBM_STEADY_TOL || end[i] == LBM_STEADY_PLATEAU;
        if (steps) steps[i] = ok ? tr[i].best_step : -1;
        if (how) how[i] = end[i];
        if (last_residual) last_residual[i] = b->last_res[i];
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_launch(lbm_batch* b, int32_t threads, int32_t bpc, int32_t graph_steps) {
    if (!b) return fail(LBM_ERR_ARG, "null batch");
    int maxnx = 0;
    for (lbm_handle* h : b->mem) maxnx = std::max(maxnx, h->p.nx);
    if (threads <= 0 || threads % 64 || threads > 1024 || threads < maxnx)
        return fail(LBM_ERR_ARG, "threads must be a multiple of 64 in [max nx, 1024]");
    if (bpc < 0 || bpc > 32)
        return fail(LBM_ERR_ARG, "blocks per compute unit must be 0 (one block per tile) or 1..32");
    if (graph_steps < 0 || (graph_steps & 1)) return fail(LBM_ERR_ARG, "graph_steps must be even");
    if (graph_steps > 0 && !b->stream)
        return fail(LBM_ERR_ARG, "graphs need a batch created on a non-default stream");
    const bool reshape = threads != b->threads;
    b->threads = threads;
    b->bpc = bpc;
    b->graph_steps = graph_steps;
    if (reshape) {
        lbm_status s = upload_table(b);
        if (s != LBM_OK) return s;
    }
    return capture_graph(b);
}

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t steps_per_trial, int32_t* out_threads,
                              int32_t* out_bpc) {
    if (!b || steps_per_trial <= 0) return fail(LBM_ERR_ARG, "bad arguments");
    int maxnx = 0;
    for (lbm_handle* h : b->mem) maxnx = std::max(maxnx, h->p.nx);
    static const int cand_t[] = {128, 192, 256, 320, 384, 512, 768, 1024};
    static const int cand_b[] = {0, 2, 4, 8, 16};  // 0: one block per tile
    const int gsteps_keep = b->graph_steps;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "autotune events");
    float best = 1e30f;
    int bt = b->threads, bb = b->bpc;
    lbm_status s = LBM_OK;
    for (int t : cand_t) {
        if (t < maxnx) continue;
        for (int bp : cand_b) {
            if (t * bp > 32 * 64 * 4) continue;  // more threads than a compute unit holds
            s = lbm_batch_set_launch(b, t, bp, 0);
            if (s != LBM_OK) break;
            s = lbm_batch_step(b, 2);
            if (s != LBM_OK) break;
            e = hipEventRecord(e0, b->stream);
            if (e == hipSuccess) s = lbm_batch_step(b, steps_per_trial);
            if (e == hipSuccess && s == LBM_OK) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess && s == LBM_OK) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess && s == LBM_OK) e = hipEventElapsedTime(&ms, e0, e1);
            if (s != LBM_OK || e != hipSuccess) break;
            if (ms < best) best = ms, bt = t, bb = bp;
        }
        if (s != LBM_OK || e != hipSuccess) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != LBM_OK) return s;
    if (e != hipSuccess) return hip_fail(e, "autotune");
    s = lbm_batch_set_launch(b, bt, bb, gsteps_keep);
    if (s != LBM_OK) return s;
    if (out_threads) *out_threads = bt;
    if (out_bpc) *out_bpc = bb;
    return LBM_OK;
}

lbm_status lbm_batch_launch_info(lbm_batch* b, int32_t* threads, int32_t* grid_blocks,
                                 int32_t* active_tiles, int32_t* graph_steps, int64_t* steps) {
    if (!b) return fail(LBM_ERR_ARG, "null batch");
    if (threads) *threads = b->threads;
    if (grid_blocks) *grid_blocks = (int32_t)batch_grid(b);
    if (graph_steps) *graph_steps = b->graph_ok ? b->graph_steps : 0;
    if (steps) *steps = b->gsteps;
    if (active_tiles) {
        uint32_t nt = 0;
        hipError_t e = hipMemcpyAsync(&nt, b->d_ntiles(), sizeof nt, hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(e, "launch info");
        *active_tiles = (int32_t)nt;
    }
    return LBM_OK;
}

}  // extern "C"

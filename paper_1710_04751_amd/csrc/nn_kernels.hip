// gfx950 kernels of the warm-start network: 3D convolutions as implicit
// GEMMs on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), the 1 x 1 x 1 head with the loss on the vector units,
// pooling, upsampling and Adam.
//
// Matrix-core fragments (64 lanes, r = lane % 16, q = lane / 16):
//   A (16 x 32): lane holds row r, k = 8q .. 8q+7;
//   B (32 x 16): lane holds column r, k = 8q .. 8q+7;
//   D (16 x 16, FP32): lane holds rows 4q .. 4q+3 of column r.
// Forward: rows are 16 voxels, columns output channels, k runs over
// (tap, input channel) with the channels of one tap contiguous, so a lane's
// 8 k values are one 16-byte load of a channels-last voxel.  The input
// gradient is the same kernel run on the output gradient with the
// transposed, tap-flipped weight.  The weight gradient takes rows = output
// channels, columns = (tap, input channel) and k = voxels; each block sums
// a range of voxels and writes its partial sums, and a second kernel adds
// the partials of all ranges in a fixed order (no atomics, so gradients are
// bit-reproducible).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "nn_internal.hpp"

namespace lbmnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_void_ptr;  // LDS destination of direct loads

namespace {

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// Per-sample scalars passed by value (at most kMaxBatch samples).
struct SampleFloats {
    float v[kMaxBatch];
};
struct SampleInts {
    int32_t v[kMaxBatch];
};

// One layer of the weight packing: destinations, the layer's offset in the
// master parameters and its geometry.
struct PackLayer {
    __bf16* wp;
    __bf16* wt;
    int64_t woff;
    int32_t coutp, kpad, cout, K, cin, c1, c1s, taps, cin_real, cinp, kpad_t, ys;
};
struct PackTable {
    PackLayer l[kMaxPackLayers];
    int64_t blk[2 * kMaxPackLayers];  // cumulative blocks of 256 over the segments
};

struct ConvArgs {
    const __bf16* x1;
    const __bf16* x2;
    const __bf16* w;
    const float* bias;
    __bf16* out;
    const __bf16* omask;  // outputs where omask <= 0 are written as 0
    int32_t n, lg, taps, c1s, c2, cin, K, kpad, cout, ys, relu;
    int32_t wrows;        // rows of the packed weight w (set by launch_conv)
};

// One block: MT * 16 voxels x (NSUB * 16) output channels, channel group
// blockIdx.y.  Each weight fragment is loaded once and used for the MT
// voxel tiles.  The KS waves of a block split the k range (wave w takes
// every KS-th step of 32 from step w) and add their partial sums through
// LDS; this keeps enough waves in flight on the coarse grids.
template <int NSUB, int MT, int KS>
__global__ void __launch_bounds__(64 * KS) k_conv(ConvArgs a) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int wave = threadIdx.x >> 6;
    const int lg = a.lg, G = 1 << lg;
    const int64_t V = (int64_t)1 << (3 * lg);
    const int64_t M = (int64_t)a.n * V;
    const int64_t vb = (int64_t)blockIdx.x * (16 * MT);
    const int cobase = blockIdx.y * NSUB * 16;
    bool vok[MT];
    int vs[MT], vz[MT], vy[MT], vx[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int64_t v = vb + m * 16 + r;
        vok[m] = v < M;
        const int64_t vc = vok[m] ? v : 0;
        vs[m] = (int)(vc >> (3 * lg));
        const int rem = (int)(vc & (V - 1));
        vz[m] = rem >> (2 * lg);
        vy[m] = (rem >> lg) & (G - 1);
        vx[m] = rem & (G - 1);
    }
    floatx4 acc[MT][NSUB];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NSUB; ++j) acc[m][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // Wave w takes the k steps w, w + KS, ...: nst of them; at step s the
    // lane's 8 k values start at kw + 32 KS s.  The fragments of a step are
    // A (MT voxel tiles, 8 channels of one tap per lane) and B (NSUB weight
    // tiles).  With one voxel tile two register sets take turns: the loads of
    // step s + 1 go into one while the matrix cores work on step s in the
    // other.  The loop body has no branches (a lane outside the grid loads
    // voxel 0 and takes zeros; a step past the last reloads the last one's
    // addresses with a zero A fragment, so its products add 0), so the
    // compiler keeps the loads ahead of the products and the waits cover
    // only the step in use.
    const int kw = q * 8 + 32 * wave;
    const int nst = kw < a.kpad ? (a.kpad - 1 - kw) / (32 * KS) + 1 : 0;
    const float icin = 1.f / (float)a.cin;
    const int h = lg - 1;
    auto load_step = [&](int st, bf16x8* av, bf16x8* bv) __attribute__((always_inline)) {
        const bool live = st < nst;
        const int k = kw + (live ? st : nst - 1) * (32 * KS);
        // tap = k / cin (exact: k < 2^13, so (k + 0.5) / cin is far from an integer)
        const int tap = (int)(((float)k + 0.5f) * icin), c = k - tap * a.cin;
        const bool t27 = a.taps == 27;
        const int dz = t27 ? tap / 9 - 1 : 0, dy = t27 ? (tap / 3) % 3 - 1 : 0,
                  dx = t27 ? tap % 3 - 1 : 0;
        const bool lo = c < a.c1s;
        const __bf16* base = lo ? a.x1 : a.x2;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int zz = vz[m] + dz, yy = vy[m] + dy, xx = vx[m] + dx;
            const bool ok = live && vok[m] && k < a.K && (unsigned)zz < (unsigned)G &&
                            (unsigned)yy < (unsigned)G && (unsigned)xx < (unsigned)G;
            const int zc = ok ? zz : 0, yc = ok ? yy : 0, xc = ok ? xx : 0;
            const int64_t off =
                lo ? (((int64_t)vs[m] << (3 * lg)) + ((int64_t)zc << (2 * lg)) +
                      ((int64_t)yc << lg) + xc) * a.c1s + c
                   : (((int64_t)vs[m] << (3 * h)) + ((int64_t)(zc >> 1) << (2 * h)) +
                      ((int64_t)(yc >> 1) << h) + (xc >> 1)) * a.c2 + (c - a.c1s);
            const bf16x8 v = *(const bf16x8*)(base + off);
#pragma unroll
            for (int i = 0; i < 8; ++i) av[m][i] = ok ? v[i] : (__bf16)0.f;
        }
#pragma unroll
        for (int j = 0; j < NSUB; ++j)
            bv[j] = *(const bf16x8*)(a.w + (int64_t)(cobase + j * 16 + r) * a.kpad + k);
    };
    auto products = [&](const bf16x8* av, const bf16x8* bv) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < NSUB; ++j)
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[j], acc[m][j], 0, 0, 0);
    };
    if constexpr (MT == 1) {
        if (nst > 0) {
            bf16x8 a0[MT], b0[NSUB], a1[MT], b1[NSUB];
            load_step(0, a0, b0);
            for (int st = 0; st < nst; st += 2) {
                load_step(st + 1, a1, b1);
                products(a0, b0);
                load_step(st + 2, a0, b0);
                products(a1, b1);
            }
        }
    } else {
        // four voxel tiles: a second register set would cost more occupancy
        // than its prefetch gains (measured), so each step loads and uses one
        for (int st = 0; st < nst; ++st) {
            bf16x8 a0[MT], b0[NSUB];
            load_step(st, a0, b0);
            products(a0, b0);
        }
    }
    if constexpr (KS > 1) {
        __shared__ floatx4 part[KS - 1][MT * NSUB][64];
        if (wave > 0) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int j = 0; j < NSUB; ++j) part[wave - 1][m * NSUB + j][lane] = acc[m][j];
        }
        __syncthreads();
        if (wave > 0) return;
#pragma unroll
        for (int w = 0; w < KS - 1; ++w)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int j = 0; j < NSUB; ++j) acc[m][j] += part[w][m * NSUB + j][lane];
    }
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t vo = vb + m * 16 + q * 4 + i;
            if (vo >= M) continue;
#pragma unroll
            for (int j = 0; j < NSUB; ++j) {
                const int co = cobase + j * 16 + r;
                if (co < a.ys) {
                    float val = 0.f;
                    if (co < a.cout) {
                        val = acc[m][j][i] + (a.bias ? a.bias[co] : 0.f);
                        if (a.relu) val = fmaxf(val, 0.f);
                        if (a.omask && !((float)a.omask[vo * a.ys + co] > 0.f)) val = 0.f;
                    }
                    a.out[vo * a.ys + co] = (__bf16)val;
                }
            }
        }
}

struct WgradArgs {
    const __bf16* x1;
    const __bf16* x2;
    const __bf16* dy;
    const __bf16* y;
    float* part;    // partial sums: weights of every block, then the bias partials
    int64_t bias_off;  // floats from part to the bias partials
    int32_t n, lg, taps, c1, c1s, c2, cin, K, cout, coutp, ys, relu, cin_real;
    int64_t vchunk;
};

// LDS layouts follow what the part's LDS serves without bank conflicts
// (measured with a probe over 768 layouts): for 16-byte reads where lane
// (r, q) = (lane % 16, lane / 16) reads byte r S + (q & 1) H + (q >> 1) T, T
// never matters; S = 16 is conflict-free for any H; S = 32 (mod 64) for H = 16
// or 48; S = 16 or 48 (mod 64) only for H a multiple of 256 (or S = H = 48);
// S = 0 (mod 64) never.  The fragments here have H = 16 (the lane's second 8
// channels or k values), so row strides are 32 (mod 64) bytes.
constexpr int kTileRow = 48;   // 32-voxel tile rows, in elements (96 bytes)
constexpr int kDTRow = 144;    // 128-voxel brick rows of the output gradient (288 bytes)

// B fragment of ones: an A fragment times it gives its row sums in every
// column (the bias gradient's sum over voxels, on the matrix cores).
__device__ __forceinline__ bf16x8 ones_frag() {
    bf16x8 o;
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = (__bf16)1.f;
    return o;
}

// Weight gradient, one block of 4 waves per (row tile, column tile, voxel
// chunk): rows are RS * 16 output channels, columns CS * 16 (tap, channel)
// pairs with RS * CS = 8, so each wave owns two 16 x 16 accumulators.  Per
// 32 voxels the block loads the masked output gradient and the input patch
// with 16-byte loads (8 channels of one voxel) and writes them transposed
// into LDS ([channel][voxel]), where each fragment (8 consecutive voxels) is
// one 16-byte read.  Blocks of the first column tile also sum the output
// gradient into the bias gradient (one more matrix-core product, against
// ones).  Every block writes its partial sums to part (block b = (z * ct +
// y) * kt + x: RS * 16 rows x CS * 16 columns; bias partials [z * ct + y][RS
// * 16] at bias_off); k_wgrad_reduce adds them up.
template <int RS>
__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a) {
    constexpr int CS = 8 / RS;
    __shared__ __attribute__((aligned(16))) __bf16 dT[RS * 16][kTileRow];
    __shared__ __attribute__((aligned(16))) __bf16 xT[CS * 16][kTileRow];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int lg = a.lg, G = 1 << lg;
    const int64_t V = (int64_t)1 << (3 * lg);
    const int64_t M = (int64_t)a.n * V;
    const int row0 = blockIdx.y * RS * 16, col0 = blockIdx.x * CS * 16;
    const int wr = wave % RS, wc = 2 * (wave / RS);
    floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    floatx4 accb = {0.f, 0.f, 0.f, 0.f};
    const bool bias_wave = blockIdx.x == 0 && wave < RS;  // wc == 0
    const int64_t v0 = (int64_t)blockIdx.z * a.vchunk;
    const int64_t v1 = std::min(M, v0 + a.vchunk);
    for (int64_t vb = v0; vb < v1; vb += 32) {
        // output gradient: RS*2 groups of 8 channels x 32 voxels
        for (int t = tid; t < RS * 2 * 32; t += 256) {
            const int g8 = t >> 5, vi = t & 31;
            const int c0 = row0 + g8 * 8;
            const int64_t vv = vb + vi;
            bf16x8 d;
#pragma unroll
            for (int i = 0; i < 8; ++i) d[i] = (__bf16)0.f;
            if (vv < v1 && c0 < a.ys) {
                d = *(const bf16x8*)(a.dy + vv * a.ys + c0);
                if (a.relu) {
                    const bf16x8 m = *(const bf16x8*)(a.y + vv * a.ys + c0);
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (!((float)m[i] > 0.f)) d[i] = (__bf16)0.f;
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) dT[g8 * 8 + i][vi] = d[i];
        }
        // input patches: CS*2 groups of 8 (tap, channel) columns x 32 voxels
        for (int t = tid; t < CS * 2 * 32; t += 256) {
            const int g8 = t >> 5, vi = t & 31;
            const int k0 = col0 + g8 * 8;
            const int64_t vv = vb + vi;
            bf16x8 xv;
#pragma unroll
            for (int i = 0; i < 8; ++i) xv[i] = (__bf16)0.f;
            if (vv < v1 && k0 < a.K) {
                const int tap = k0 / a.cin, c = k0 - tap * a.cin;
                const int s = (int)(vv >> (3 * lg));
                const int rem = (int)(vv & (V - 1));
                int z = rem >> (2 * lg), y = (rem >> lg) & (G - 1), x = rem & (G - 1);
                if (a.taps == 27) {
                    z += tap / 9 - 1;
                    y += (tap / 3) % 3 - 1;
                    x += tap % 3 - 1;
                }
                if ((unsigned)z < (unsigned)G && (unsigned)y < (unsigned)G &&
                    (unsigned)x < (unsigned)G) {
                    if (c < a.c1s) {
                        const int64_t vi2 = ((int64_t)s << (3 * lg)) + ((int64_t)z << (2 * lg)) +
                                            ((int64_t)y << lg) + x;
                        xv = *(const bf16x8*)(a.x1 + vi2 * a.c1s + c);
                    } else {
                        const int h = lg - 1;
                        const int64_t vi2 = ((int64_t)s << (3 * h)) +
                                            ((int64_t)(z >> 1) << (2 * h)) +
                                            ((int64_t)(y >> 1) << h) + (x >> 1);
                        xv = *(const bf16x8*)(a.x2 + vi2 * a.c2 + (c - a.c1s));
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) xT[g8 * 8 + i][vi] = xv[i];
        }
        __syncthreads();
        const bf16x8 av = *(const bf16x8*)&dT[wr * 16 + r][q * 8];
        const bf16x8 b0 = *(const bf16x8*)&xT[wc * 16 + r][q * 8];
        const bf16x8 b1 = *(const bf16x8*)&xT[(wc + 1) * 16 + r][q * 8];
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b1, acc1, 0, 0, 0);
        if (bias_wave) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones_frag(), accb, 0, 0, 0);
        __syncthreads();
    }
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float* pb = a.part + blk * (RS * 16) * (CS * 16);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const floatx4 acc = j ? acc1 : acc0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            pb[(wr * 16 + q * 4 + i) * (CS * 16) + (wc + j) * 16 + r] = acc[i];
    }
    if (bias_wave && r == 0) {
        float* bb = a.part + a.bias_off + ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * (RS * 16);
#pragma unroll
        for (int i = 0; i < 4; ++i) bb[wr * 16 + q * 4 + i] = accb[i];
    }
}

// First pass of the partial-sum reduction: for the weight partials (rows x
// ww floats at in) and then the bias partials (rows x bw floats at in +
// boff), out[j][w] = sum of in[g][w] over the rows g of slice j (kRowSlice
// consecutive rows, fewer in the last), in order.  One thread per (slice,
// column), so the loads of many rows are in flight at once; the weight
// slices go to out, the bias slices after them.
constexpr int kRowSlice = 16;
__global__ void k_sum_row_slices(const float* __restrict__ in, int64_t boff, int64_t rows,
                                 int64_t ww, int64_t bw, float* __restrict__ out) {
    const int64_t slices = (rows + kRowSlice - 1) / kRowSlice;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t width = ww;
    if (i >= slices * ww) {
        i -= slices * ww;
        if (i >= slices * bw) return;
        in += boff;
        out += slices * ww;
        width = bw;
    }
    const int64_t j = i / width, w = i - j * width;
    const int64_t g0 = j * kRowSlice;
    const int n = (int)(rows - g0 < kRowSlice ? rows - g0 : kRowSlice);
    float v[kRowSlice];
#pragma unroll
    for (int k = 0; k < kRowSlice; ++k) v[k] = k < n ? in[(g0 + k) * width + w] : 0.f;
    float sum = 0.f;
#pragma unroll
    for (int k = 0; k < kRowSlice; ++k) sum += v[k];
    out[i] = sum;
}

// Sum over the rows of a partial-sum table by L consecutive lanes per
// gradient entry (L = 8 for tables of many rows, 1 for few): lane j adds rows
// j, j + L, ... in order, then a fixed xor butterfly adds the L lane sums
// (lane 0's result is written), so the order of every addition is fixed and,
// for many rows, many loads are in flight.
template <int L>
__device__ __forceinline__ float lane_group_sum(float v) {
    if constexpr (L >= 2) v += __shfl_xor(v, 1, L);
    if constexpr (L >= 4) v += __shfl_xor(v, 2, L);
    if constexpr (L >= 8) v += __shfl_xor(v, 4, L);
    return v;
}
constexpr int kRedManyRows = 32;  // rows from which a table takes 8 lanes per entry

// Sum of the k_wgrad partials over the voxel chunks, into the master layout
// dw[co][tap][ci] (zero padding channels dropped) and db.  One group of L
// lanes per (row, column) of the gradient matrix or per bias entry.
template <int L>
__global__ void k_wgrad_reduce(WgradArgs a, int kt, int ct, int nz, int rs, int cs, float* dw,
                               float* db) {
    // 32-bit index arithmetic: the host launches fewer than 2^31 lanes
    const uint32_t rows = (uint32_t)(ct * rs * 16), cols = (uint32_t)(kt * cs * 16);
    const uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) / L;
    const int j = threadIdx.x % L;
    if (i < rows * cols) {
        const uint32_t row = i / cols, col = i - row * cols;
        const uint32_t cty = row / (uint32_t)(rs * 16), rl = row - cty * (uint32_t)(rs * 16);
        const uint32_t ktx = col / (uint32_t)(cs * 16), cl = col - ktx * (uint32_t)(cs * 16);
        if (row >= (uint32_t)a.cout || col >= (uint32_t)a.K) return;
        const uint32_t t = col / (uint32_t)a.cin, cc = col - t * (uint32_t)a.cin;
        if (cc < (uint32_t)a.c1s && cc >= (uint32_t)a.c1) return;  // zero padding channels of x1
        const uint32_t ci = cc < (uint32_t)a.c1s ? cc : a.c1 + (cc - a.c1s);
        const int64_t per = (int64_t)rs * 16 * cs * 16;
        float sum = 0.f;
#pragma unroll 4
        for (int z = j; z < nz; z += L)
            sum += a.part[(((int64_t)z * ct + cty) * kt + ktx) * per + rl * (cs * 16) + cl];
        sum = lane_group_sum<L>(sum);
        if (j == 0) dw[((int64_t)row * a.taps + t) * a.cin_real + ci] = sum;
    } else if (i < rows * cols + (uint32_t)a.cout) {
        const uint32_t co = i - rows * cols;
        const uint32_t cty = co / (uint32_t)(rs * 16), rl = co - cty * (uint32_t)(rs * 16);
        float sum = 0.f;
        for (int z = j; z < nz; z += L)
            sum += a.part[a.bias_off + ((int64_t)z * ct + cty) * (rs * 16) + rl];
        sum = lane_group_sum<L>(sum);
        if (j == 0) db[co] = sum;
    }
}

// Weight gradient on voxel bricks, for grids of at least 16 cells and
// unmasked output gradients.  One block of 4 waves owns 16 input channels
// (blockIdx.x) and every tap and output channel (RS * 16); it walks a range
// of bricks of 16 x 4 x 2 voxels, four matrix-core k steps of 32 voxels (two
// x rows of one plane each).  Per brick:
//   - the input's 18 x 6 x 4 halo is loaded once: a thread takes 10
//     consecutive x cells of one row and 8 channels (16-byte loads),
//     transposes them in registers and writes, for dx = -1, 0, +1, the 8
//     cells each shift needs as one 16-byte LDS store per channel, so the B
//     fragment of every tap (8 consecutive cells of one channel) is one
//     aligned 16-byte read;
//   - the output gradient is transposed the same way (8 cells x 8 channels
//     per thread), and its A fragments serve all taps.
// Wave w accumulates taps w, w + 4, ...  Each block writes its partial sums
// (block b = blockIdx.y * gridDim.x + blockIdx.x: [tap][co][16 channels]);
// wave 0 of the first channel group also sums the output gradient for the
// bias (a matrix-core product against ones; partials [blockIdx.y][coutp] at
// bias_off).  k_brick_partials_sum adds the partials up.
constexpr int kBrickRow = 4 * 6 * 16 + 16;  // one channel's halo (hz, hy, x), padded

template <int RS>
__global__ void __launch_bounds__(256, 2) k_wgrad_brick(WgradArgs a, int64_t bricks_per_block) {
    constexpr int NT = 7;  // taps per wave: ceil(27 / 4)
    __shared__ __attribute__((aligned(16))) __bf16 xs[3 * 16 * kBrickRow];
    __shared__ __attribute__((aligned(16))) __bf16 dT[RS * 16][kDTRow];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int lg = a.lg, G = 1 << lg;
    const int c0 = blockIdx.x * 16;
    const int nbx = G >> 4, nby = G >> 2, nbz = G >> 1;
    const int64_t nbricks = (int64_t)a.n * nbz * nby * nbx;
    const int64_t b0 = (int64_t)blockIdx.y * bricks_per_block;
    const int64_t b1 = b0 + bricks_per_block < nbricks ? b0 + bricks_per_block : nbricks;
    floatx4 acc[NT][RS];
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int m = 0; m < RS; ++m) acc[j][m] = floatx4{0.f, 0.f, 0.f, 0.f};
    floatx4 accb[RS];
#pragma unroll
    for (int m = 0; m < RS; ++m) accb[m] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bool bias_wave = blockIdx.x == 0 && wave == 0;
    // Roles: threads 0-95 load input halo rows, the next 32 * RS the output
    // gradient.  The global loads of brick b + 1 are issued into registers
    // before the matrix-core phase of brick b, so their latency is hidden.
    const int cgx = tid / 48, remx = tid - cgx * 48;
    const int kx = remx & 1, hyx = (remx >> 1) % 6, hzx = (remx >> 1) / 6;
    const int td = tid - 96, vgd = td & 15, cgd = td >> 4, sd = vgd >> 2;
    // Loads through range-checked buffer resources over one sample of the
    // channel group's tensor and of the output gradient (zeros past the end:
    // no branch, select or zero fill, so no load waits on another).
    const int h = lg - 1;
    const bool lo = c0 < a.c1s;
    const int chans = lo ? a.c1s : a.c2;
    const int hl = lo ? lg : h;
    const int64_t vs = (int64_t)1 << (3 * hl);
    const uint32_t xbytes = (uint32_t)(vs * chans * 2);
    const uint32_t dbytes = (uint32_t)(((int64_t)1 << (3 * lg)) * a.ys * 2);
    const int cloc = lo ? c0 : c0 - a.c1s;
    bf16x8 reg[10];
    auto fetch = [&](int64_t b) __attribute__((always_inline)) {
        uint32_t bb = (uint32_t)b;
        const int x0 = (int)(bb % (uint32_t)nbx) * 16;
        bb /= (uint32_t)nbx;
        const int y0 = (int)(bb % (uint32_t)nby) * 4;
        bb /= (uint32_t)nby;
        const int z0 = (int)(bb % (uint32_t)nbz) * 2;
        const int smp = (int)(bb / (uint32_t)nbz);
        if (tid < 96) {
            // input halo row (hz, hy), x cells 8k .. 8k+9, channel group cg
            // (the channel group is the slowest index)
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<__bf16*>((lo ? a.x1 : a.x2) + (int64_t)smp * vs * chans), (short)0,
                (int)xbytes, 0x00020000);
            const int yy = y0 + hyx - 1, zz = z0 + hzx - 1;
            const bool row_ok = c0 + cgx * 8 < a.cin && (unsigned)yy < (unsigned)G &&
                                (unsigned)zz < (unsigned)G;
            const int sh = lo ? 0 : 1;
            const uint32_t rowv = ((uint32_t)(zz >> sh) << (2 * hl)) + ((uint32_t)(yy >> sh) << hl);
#pragma unroll
            for (int m = 0; m < 10; ++m) {
                const int xx = x0 + 8 * kx + m - 1;
                const bool ok = row_ok && (unsigned)xx < (unsigned)G;
                const uint32_t off =
                    (((rowv + (uint32_t)(xx >> sh)) * (uint32_t)chans + (uint32_t)(cloc + cgx * 8)) * 2u) |
                    ((uint32_t)!ok << 31);
                reg[m] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
            }
        } else if (tid < 96 + 32 * RS) {
            // output gradient: 8 cells (one k group) x 8 channels
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<__bf16*>(a.dy + ((int64_t)smp << (3 * lg)) * a.ys), (short)0,
                (int)dbytes, 0x00020000);
            const int yy = y0 + (sd & 1) * 2 + ((vgd & 3) >> 1), zz = z0 + (sd >> 1);
            const int xb = x0 + (vgd & 1) * 8;
            const uint32_t v0 = ((uint32_t)zz << (2 * lg)) + ((uint32_t)yy << lg) + (uint32_t)xb;
            const uint32_t bad = (uint32_t)!(cgd * 8 < a.ys) << 31;
#pragma unroll
            for (int m = 0; m < 8; ++m)
                reg[m] = __builtin_bit_cast(
                    bf16x8, __builtin_amdgcn_raw_buffer_load_b128(
                                rs, (((v0 + m) * (uint32_t)a.ys + (uint32_t)(cgd * 8)) * 2u) | bad,
                                0, 0));
        }
    };
    if (b0 < b1) fetch(b0);
    for (int64_t b = b0; b < b1; ++b) {
        // transposed LDS stores of the fetched brick
        if (tid < 96) {
            const int row = (hzx * 6 + hyx) * 16 + 8 * kx;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    bf16x8 w;
#pragma unroll
                    for (int j = 0; j < 8; ++j) w[j] = reg[j + d][e];
                    *(bf16x8*)&xs[(d * 16 + cgx * 8 + e) * kBrickRow + row] = w;
                }
        } else if (tid < 96 + 32 * RS) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                bf16x8 w;
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = reg[j][e];
                *(bf16x8*)&dT[cgd * 8 + e][vgd * 8] = w;
            }
        }
        __syncthreads();
        if (b + 1 < b1) fetch(b + 1);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            bf16x8 av[RS];
#pragma unroll
            for (int m = 0; m < RS; ++m) av[m] = *(const bf16x8*)&dT[m * 16 + r][s * 32 + q * 8];
            if (bias_wave) {
#pragma unroll
                for (int m = 0; m < RS; ++m)
                    accb[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], ones_frag(), accb[m],
                                                                      0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int t = wave + 4 * j;
                if (t < 27) {
                    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
                    const int hz = (s >> 1) + dz + 1, hy = (s & 1) * 2 + (q >> 1) + dy + 1;
                    const bf16x8 bv = *(const bf16x8*)&xs[((dx + 1) * 16 + r) * kBrickRow +
                                                          (hz * 6 + hy) * 16 + (q & 1) * 8];
#pragma unroll
                    for (int m = 0; m < RS; ++m)
                        acc[j][m] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv, acc[j][m], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    float* pb = a.part + blk * (27 * RS * 16 * 16);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int t = wave + 4 * j;
        if (t >= 27) continue;
#pragma unroll
        for (int m = 0; m < RS; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                pb[((t * RS + m) * 16 + q * 4 + i) * 16 + r] = acc[j][m][i];
    }
    if (bias_wave && r == 0) {
        float* bb = a.part + a.bias_off + (int64_t)blockIdx.y * (RS * 16);
#pragma unroll
        for (int m = 0; m < RS; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) bb[m * 16 + q * 4 + i] = accb[m][i];
    }
}

// Weight gradient on 16 x 4 x 4 bricks through transposing LDS reads, for
// 16 and 32 output channels.  dW[tap][co][ci] sums dY[v][co] X[v + tap][ci]
// over voxels v, so both matrix-core operands need 8 consecutive voxels of one
// channel per lane, while the tensors are stored channels-last.  The block
// copies the brick's output gradient and the 18 x 6 x 6 input halo of one
// 16-channel group into LDS as they are stored (direct-to-LDS loads, 32 bytes
// per voxel and 16 channels), and ds_read_b64_tr_b16 transposes on the way
// out: within each 16 lanes, lane 4a + b receives element b of the 8-byte
// pieces addressed by lanes a, a + 4, a + 8, a + 12.  So when lane L of a
// group addresses voxel k0 + L / 4, channels 4 (L % 4) .. + 3, lane n gets
// voxels k0 .. k0 + 3 of channel n: two such reads give an operand fragment.
// Nine waves, wave w the three taps with dz = w / 3 - 1, dy = w % 3 - 1.  Lane
// groups q and q ^ 1 of a k step take neighbouring rows, and the LDS rows are
// padded so that their reads fall in opposite halves of the banks (a row of
// the halo or of a one-group output gradient holds 20 voxels, 640 bytes; of a
// two-group output gradient 1056 bytes).  A block walks a range of bricks in
// z order within each (x, y) column; the halo is a ring of 8 plane slots
// (input plane z in slot z mod 8), so a brick that follows its z neighbour
// keeps the two planes they share and copies only its 4 new ones.  Partial
// sums as k_wgrad_brick.
constexpr int kWtWaves = 9;
constexpr int kWtHaloRow = 20;                 // voxels per LDS halo row (18 + 2 padding)
constexpr int kWtPlaneItems = 256;             // 16-byte items per plane slot: 6 rows, padding
constexpr int kWtRing = 8;                     // plane slots
constexpr int kWtHaloBuf = kWtRing * kWtPlaneItems;
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) shortx4* lds_shortx4_ptr;

__device__ __forceinline__ bf16x8 tr_fragment(const char* lds, uint32_t byte0, uint32_t byte1) {
    const shortx4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_shortx4_ptr)(lds + byte0));
    const shortx4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_shortx4_ptr)(lds + byte1));
    return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <int RS>
__global__ void __launch_bounds__(64 * kWtWaves) k_wgrad_tr(WgradArgs a, int64_t bricks_per_block) {
    constexpr int kDyRow = RS == 1 ? 40 : 66;   // 16-byte items per output-gradient row (padded)
    constexpr int kDyItems = 16 * kDyRow;       // 4 planes x 4 rows
    constexpr int kDyBuf = (kDyItems + 63) / 64 * 64;
    constexpr int kDyCopies = kDyBuf / 64;
    constexpr int kDyByte = kWtHaloBuf * 16;  // byte offset of the output gradient in LDS
    constexpr int kMaxCopies = 6 * kWtPlaneItems / 64 + kDyCopies;  // a brick with a new halo
    __shared__ __attribute__((aligned(16))) __bf16 set[(kWtHaloBuf + kDyBuf) * 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int lg = a.lg, G = 1 << lg;
    // XCD-grouped order: the dispatcher deals consecutive blocks to the 8 XCDs
    // in turn, so logical block (lin mod 8) (total / 8) + lin / 8 puts runs of
    // consecutive (range, channel group) pairs on one XCD: the channel groups
    // of a range share its output gradient, neighbouring ranges their halo
    // rows, in that XCD's L2
    const uint32_t total = gridDim.x * gridDim.y, lin = blockIdx.y * gridDim.x + blockIdx.x;
    const uint32_t lblk = total % 8 ? lin : (lin % 8) * (total / 8) + lin / 8;
    const int chunk = (int)(lblk % gridDim.x), grp = (int)(lblk / gridDim.x);
    const int c0 = chunk * 16;
    const int nbx = G >> 4, nby = G >> 2, nbz = G >> 2;
    const int64_t nbricks = (int64_t)a.n * nbz * nby * nbx;
    const int64_t b0 = (int64_t)grp * bricks_per_block;
    const int64_t b1 = b0 + bricks_per_block < nbricks ? b0 + bricks_per_block : nbricks;
    floatx4 acc[3][RS];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int m = 0; m < RS; ++m) acc[j][m] = floatx4{0.f, 0.f, 0.f, 0.f};
    floatx4 accb[RS];
#pragma unroll
    for (int m = 0; m < RS; ++m) accb[m] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bool bias_wave = chunk == 0 && wave == 0;
    // k value 8 q + 4 h + e of k step s (h: which of the two reads, e = r / 4)
    // is the brick voxel (plane s / 2, row 2 (s % 2) + q % 2, cell 8 (q / 2) +
    // 4 h + e); the lane reads channels 4 (r % 4) .. + 3 of it
    const int e = r >> 2, ac = r & 3;
    const uint32_t laneA =
        (uint32_t)(kDyByte + ((q & 1) * kDyRow + (8 * (q >> 1) + e) * 2 * RS) * 16 + ac * 8);
    const int dzw = wave / 3, dyw = wave % 3;  // this wave's taps: dz + 1, dy + 1
    // within a plane slot (the slot's offset is added per brick)
    const uint32_t laneB = (uint32_t)((((q & 1) + dyw) * kWtHaloRow + 8 * (q >> 1) + e) * 32 + ac * 8);
    const int h = lg - 1;
    const bool lo = c0 < a.c1s;  // the group's channels lie in x1 (else x2; c1s is then a multiple of 16)
    const int chans = lo ? a.c1s : a.c2;
    const int hl = lo ? lg : h, sh = lo ? 0 : 1;
    const int64_t vs = (int64_t)1 << (3 * hl);
    const int cloc = lo ? c0 : c0 - a.c1s;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // brick b: z fastest, then x, y, sample
    auto brick = [&](int64_t b, int& x0, int& y0, int& z0, int& smp) __attribute__((always_inline)) {
        uint32_t bb = (uint32_t)b;
        z0 = (int)(bb % (uint32_t)nbz) * 4;
        bb /= (uint32_t)nbz;
        x0 = (int)(bb % (uint32_t)nbx) * 16;
        bb /= (uint32_t)nbx;
        y0 = (int)(bb % (uint32_t)nby) * 4;
        smp = (int)(bb / (uint32_t)nby);
    };
    // The copies of brick b: the halo planes z0 - 1 .. z0 + 4 when the brick
    // starts a run (the block's first, or the first of its column), else
    // z0 + 1 .. z0 + 4 (the other two are in the ring from the brick before);
    // then the output gradient.  Copy j goes to wave j % 9.
    auto issue = [&](int64_t b) __attribute__((always_inline)) {
        int x0, y0, z0, smp;
        brick(b, x0, y0, z0, smp);
        const bool fresh = b == b0 || z0 == 0;
        const int zfirst = fresh ? z0 - 1 : z0 + 1;
        const int nh = (fresh ? 6 : 4) * (kWtPlaneItems / 64);  // halo copies
        const int ncopies = nh + kDyCopies;
        // range-checked buffer resources: positions outside the grid, channel
        // halves past the input channels, output channels past ys and padding
        // items read zeros
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<__bf16*>((lo ? a.x1 : a.x2) + (int64_t)smp * vs * chans), (short)0,
            (int)(uint32_t)(vs * chans * 2), 0x00020000);
        const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<__bf16*>(a.dy + ((int64_t)smp << (3 * lg)) * a.ys), (short)0,
            (int)(uint32_t)(((int64_t)1 << (3 * lg)) * a.ys * 2), 0x00020000);
        // (the lane's item decode is redone per brick rather than held in registers)
        int ln = lane;
        __asm__ volatile("" : "+v"(ln));
#pragma unroll
        for (int i = 0; i < (kMaxCopies + kWtWaves - 1) / kWtWaves; ++i) {
            const int j = i * kWtWaves + wv;
            if (j >= ncopies) break;
            if (j < nh) {
                // halo plane zz = zfirst + j / 4 into slot zz mod 8; item t of
                // the plane: slot t / 2 of 20 x 6 (t >= 240 pads), channel half t % 2
                const int zz = zfirst + (j >> 2);
                const int t = (j & 3) * 64 + ln;
                const int half = t & 1, hv = t >> 1;
                const int hx = hv % kWtHaloRow, hy = hv / kWtHaloRow;
                const int xx = x0 + hx - 1, yy = y0 + hy - 1;
                const bool ok = hy < 6 && hx < 18 && c0 + half * 8 < a.cin &&
                                (unsigned)xx < (unsigned)G && (unsigned)yy < (unsigned)G &&
                                (unsigned)zz < (unsigned)G;
                const uint32_t vox = ((uint32_t)(zz >> sh) << (2 * hl)) +
                                     ((uint32_t)(yy >> sh) << hl) + (uint32_t)(xx >> sh);
                const uint32_t off = ((vox * (uint32_t)chans + (uint32_t)(cloc + half * 8)) * 2u) |
                                     ((uint32_t)!ok << 31);
                const int dst = (zz & (kWtRing - 1)) * kWtPlaneItems + (j & 3) * 64;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_void_ptr)&set[dst * 8], 16, off, 0, 0, 0);
            } else {
                // output-gradient item t: row t / kDyRow (4 plane + row), voxel
                // and 8 channels of item t % kDyRow (the last items of a row
                // pad); past the output gradient, padding
                const int t = (j - nh) * 64 + ln;
                const int row = t / kDyRow, it = t - row * kDyRow;
                const int px = it / (2 * RS), c8 = it % (2 * RS);
                const uint32_t vox = ((uint32_t)(z0 + ((row >> 2) & 3)) << (2 * lg)) +
                                     ((uint32_t)(y0 + (row & 3)) << lg) + (uint32_t)(x0 + (px & 15));
                const bool ok = t < kDyItems && px < 16 && c8 * 8 < a.ys;
                const uint32_t off = ((vox * (uint32_t)a.ys + (uint32_t)(c8 * 8)) * 2u) |
                                     ((uint32_t)!ok << 31);
                const int dst = kWtHaloBuf + (j - nh) * 64;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rd, (lds_void_ptr)&set[dst * 8], 16, off, 0, 0, 0);
            }
        }
    };
    // products of brick b: k step s reads halo plane z0 - 1 + s / 2 + dz + 1
    auto products = [&](int64_t b) __attribute__((always_inline)) {
        const char* sb = (const char*)set;
        const int z0 = (int)((uint32_t)b % (uint32_t)nbz) * 4;
        uint32_t bp[4];  // the lane's base in the slot of the plane of steps 2 p, 2 p + 1
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            bp[p] = laneB + (uint32_t)(((z0 - 1 + dzw + p) & (kWtRing - 1)) * kWtPlaneItems * 16);
            __asm__ volatile("" : "+v"(bp[p]));
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int ra = ((s >> 1) * 4 + 2 * (s & 1)) * kDyRow * 16;  // the step's first row
            const int vb = 2 * (s & 1) * kWtHaloRow;  // slot of the step's first cell in its plane
            bf16x8 av[RS];
#pragma unroll
            for (int m = 0; m < RS; ++m)
                av[m] = tr_fragment(sb, laneA + ra + m * 32, laneA + ra + 4 * 32 * RS + m * 32);
            if (bias_wave) {
#pragma unroll
                for (int m = 0; m < RS; ++m)
                    accb[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], ones_frag(), accb[m], 0, 0, 0);
            }
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const uint32_t base = bp[s >> 1];
                const bf16x8 bv = tr_fragment(sb, base + (vb + dx) * 32, base + (vb + dx + 4) * 32);
#pragma unroll
                for (int m = 0; m < RS; ++m)
                    acc[dx][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv, acc[dx][m], 0, 0, 0);
            }
        }
    };
    for (int64_t b = b0; b < b1; ++b) {
        issue(b);
        __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));  // vmcnt 0: this wave's copies landed
        __syncthreads();
        products(b);
        __syncthreads();
    }
    const int64_t blk = (int64_t)grp * gridDim.x + chunk;
    float* pb = a.part + blk * (27 * RS * 16 * 16);
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const int t = wave * 3 + dx;
#pragma unroll
        for (int m = 0; m < RS; ++m)
#pragma unroll
            for (int k = 0; k < 4; ++k) pb[((t * RS + m) * 16 + q * 4 + k) * 16 + r] = acc[dx][m][k];
    }
    if (bias_wave && r == 0) {
        float* bb = a.part + a.bias_off + (int64_t)grp * (RS * 16);
#pragma unroll
        for (int m = 0; m < RS; ++m)
#pragma unroll
            for (int k = 0; k < 4; ++k) bb[m * 16 + q * 4 + k] = accb[m][k];
    }
}

// Weight gradient on grids of 8 cells (the bottleneck layers), by the
// transposing LDS reads of k_wgrad_tr: a block takes one sample, one
// 16-channel input group and 32 output channels, copies the sample's
// 10 x 10 x 10 input halo (rows padded to 12 voxels) and the 32 channels of
// its output gradient (rows of 8 voxels padded to 544 bytes) into LDS, and
// nine waves (wave w the taps with dz = w / 3 - 1, dy = w % 3 - 1) walk the
// 16 k steps of 32 voxels (plane s / 2, rows 4 (s % 2) + q for lane group q).
// Partials per (sample, input group): the layout k_brick_partials_sum adds up
// (samples as its rows).
constexpr int kWsHaloRow = 12;                       // voxels per padded halo row
constexpr int kWsHaloItems = 2 * kWsHaloRow * 10 * 10;  // 2400
constexpr int kWsHaloBuf = 38 * 64;                  // whole waves
constexpr int kWsDyRow = 34;                         // 16-byte items per output-gradient row
constexpr int kWsDyItems = 64 * kWsDyRow;            // 2176 = 34 waves
constexpr int kWsCopies = (kWsHaloBuf + kWsDyItems) / 64 / kWtWaves;  // 8 per wave

__global__ void __launch_bounds__(64 * kWtWaves) k_wgrad_small(WgradArgs a) {
    static_assert((kWsHaloBuf + kWsDyItems) / 64 == kWsCopies * kWtWaves, "uniform copies");
    __shared__ __attribute__((aligned(16))) __bf16 set[(kWsHaloBuf + kWsDyItems) * 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int chunk = blockIdx.x, smp = blockIdx.y, cp = blockIdx.z;
    const int c0 = chunk * 16;
    const int rsg = a.coutp / 16;  // output-channel tiles of the layer
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<__bf16*>(a.x1 + (int64_t)smp * 512 * a.c1s), (short)0, 512 * a.c1s * 2, 0x00020000);
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<__bf16*>(a.dy + (int64_t)smp * 512 * a.ys), (short)0, 512 * a.ys * 2, 0x00020000);
#pragma unroll
    for (int j = 0; j < kWsCopies; ++j) {
        const int tb = (j * kWtWaves + wv) * 64;
        const int t0 = tb + lane;
        uint32_t off;
        __amdgpu_buffer_rsrc_t rsrc;
        if (tb < kWsHaloBuf) {
            // halo item t: slot t / 2 of 12 x 10 x 10, channel half t % 2
            const int half = t0 & 1, hv = t0 >> 1;
            const int hx = hv % kWsHaloRow, hy = (hv / kWsHaloRow) % 10, hz = hv / (10 * kWsHaloRow);
            const int xx = hx - 1, yy = hy - 1, zz = hz - 1;
            const bool ok = t0 < kWsHaloItems && hx < 10 && c0 + half * 8 < a.cin && (unsigned)xx < 8u &&
                            (unsigned)yy < 8u && (unsigned)zz < 8u;
            const uint32_t vox = ((uint32_t)zz << 6) + ((uint32_t)yy << 3) + (uint32_t)xx;
            off = ((vox * (uint32_t)a.c1s + (uint32_t)(c0 + half * 8)) * 2u) | ((uint32_t)!ok << 31);
            rsrc = rx;
        } else {
            // output-gradient item t: row t / 34 (8 z + y), voxel and 8 channels of item t % 34
            const int t = t0 - kWsHaloBuf;
            const int row = t / kWsDyRow, it = t - row * kWsDyRow;
            const int px = it >> 2, c8 = it & 3;
            const int co = cp * 32 + c8 * 8;
            const bool ok = it < 32 && co < a.ys;
            const uint32_t vox = ((uint32_t)row << 3) + (uint32_t)(px & 7);
            off = ((vox * (uint32_t)a.ys + (uint32_t)co) * 2u) | ((uint32_t)!ok << 31);
            rsrc = rd;
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_ptr)&set[tb * 8], 16, off, 0, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));  // vmcnt 0: this wave's copies landed
    __syncthreads();
    floatx4 acc[3][2], accb[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        accb[m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[d][m] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    const bool bias_wave = chunk == 0 && wave == 0;
    const int e = r >> 2, ac = r & 3;
    const int dzw = wave / 3, dyw = wave % 3;
    const uint32_t laneA = (uint32_t)(kWsHaloBuf * 16 + (q * kWsDyRow + e * 4) * 16 + ac * 8);
    const uint32_t laneB = (uint32_t)(((q + dyw) * kWsHaloRow + dzw * 10 * kWsHaloRow + e) * 32 + ac * 8);
    const char* sb = (const char*)set;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int ra = ((s >> 1) * 8 + 4 * (s & 1)) * kWsDyRow * 16;  // the step's first row
        const int vb = ((s >> 1) * 10 + 4 * (s & 1)) * kWsHaloRow;   // halo slot of its first cell
        bf16x8 av[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) av[m] = tr_fragment(sb, laneA + ra + m * 32, laneA + ra + 4 * 64 + m * 32);
        if (bias_wave) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
                accb[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], ones_frag(), accb[m], 0, 0, 0);
        }
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const bf16x8 bv = tr_fragment(sb, laneB + (vb + dx) * 32, laneB + (vb + dx + 4) * 32);
#pragma unroll
            for (int m = 0; m < 2; ++m)
                acc[dx][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv, acc[dx][m], 0, 0, 0);
        }
    }
    const int chunks = gridDim.x;
    float* pb = a.part + ((int64_t)smp * chunks + chunk) * (27 * rsg * 256);
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const int t = wave * 3 + dx;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                pb[((t * rsg + cp * 2 + m) * 16 + q * 4 + k) * 16 + r] = acc[dx][m][k];
    }
    if (bias_wave && r == 0) {
        float* bb = a.part + a.bias_off + (int64_t)smp * a.coutp + cp * 32;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int k = 0; k < 4; ++k) bb[m * 16 + q * 4 + k] = accb[m][k];
    }
}

// Sum of the brick kernels' partials over the brick ranges in one pass, into
// dw[co][tap][ci] (zero padding channels dropped) and db.  A block takes E
// entries (consecutive in a partial row) and L row lanes: lane j adds rows j,
// j + L, ... in order, then a fixed tree adds the L lane sums, so every sum
// has one fixed order.  Blocks past the weight entries take the bias.  Tables
// of few rows take L = 1 (256 entries a block, each thread its entry's rows
// in order, several loads in flight), tall ones that give fewer than two
// blocks per CU L = 32 (32 entries, 128 bytes of a row), the rest L = 8.
constexpr int kPsShortRows = 32, kPsTallRows = 256, kPsFewBlocks = 512;

template <int kPsLanes, int kEnt>
__global__ void __launch_bounds__(kEnt * kPsLanes)
k_brick_partials_sum(WgradArgs a, int chunks, int rows, int rs, float* dw, float* db) {
    const uint32_t per = (uint32_t)(27 * rs * 16 * 16);  // entries of one channel group
    const uint32_t W = per * (uint32_t)chunks;           // weight entries of a row
    const uint32_t nbw = (W + kEnt - 1) / kEnt;
    const int el = threadIdx.x % kEnt, j = threadIdx.x / kEnt;
    const bool bias = blockIdx.x >= nbw;
    const uint32_t e = (bias ? blockIdx.x - nbw : blockIdx.x) * kEnt + el;
    const bool valid = bias ? e < (uint32_t)a.cout : e < W;
    const float* base = bias ? a.part + a.bias_off : a.part;
    const uint32_t stride = bias ? (uint32_t)(rs * 16) : W;
    float v = 0.f;
    if constexpr (kPsLanes == 1) {
        if (!valid) return;
#pragma unroll 8
        for (int g = 0; g < rows; ++g) v += base[(int64_t)g * stride + e];
    } else {
        __shared__ float red[kPsLanes][kEnt + 1];
        float sum = 0.f;
        if (valid) {
#pragma unroll 4
            for (int g = j; g < rows; g += kPsLanes) sum += base[(int64_t)g * stride + e];
        }
        red[j][el] = sum;
        __syncthreads();
#pragma unroll
        for (int h = kPsLanes / 2; h > 0; h >>= 1) {
            if (j < h) red[j][el] += red[j + h][el];
            __syncthreads();
        }
        if (j != 0 || !valid) return;
        v = red[0][el];
    }
    if (bias) {
        db[e] = v;
        return;
    }
    const uint32_t chunk = e / per, r0 = e - chunk * per;
    const uint32_t t = r0 / (uint32_t)(rs * 256), rem = r0 - t * (uint32_t)(rs * 256);
    const uint32_t co = rem >> 4, cc = chunk * 16 + (rem & 15);
    if (co >= (uint32_t)a.cout || cc >= (uint32_t)a.cin || (cc < (uint32_t)a.c1s && cc >= (uint32_t)a.c1))
        return;
    const uint32_t ci = cc < (uint32_t)a.c1s ? cc : a.c1 + (cc - a.c1s);
    dw[((int64_t)co * 27 + t) * a.cin_real + ci] = v;
}

// Packed weight element idx of wp[coutp][kpad] (k = tap * cin + stored
// channel; zero padding channels and k >= K hold 0).
__device__ __forceinline__ float pack_w_elem(const PackLayer& L, int64_t idx,
                                             const float* __restrict__ w) {
    const int co = (int)(idx / L.kpad), k = (int)(idx - (int64_t)co * L.kpad);
    if (co >= L.cout || k >= L.K) return 0.f;
    const int t = k / L.cin, cc = k - t * L.cin;
    if (cc < L.c1s) return cc < L.c1 ? w[((int64_t)co * L.taps + t) * L.cin_real + cc] : 0.f;
    return w[((int64_t)co * L.taps + t) * L.cin_real + L.c1 + (cc - L.c1s)];
}

// Transposed, tap-flipped element idx of wt[cinp][kpad_t] (k = tap * ys + co).
__device__ __forceinline__ float pack_wt_elem(const PackLayer& L, int64_t idx,
                                              const float* __restrict__ w) {
    const int ci = (int)(idx / L.kpad_t), k = (int)(idx - (int64_t)ci * L.kpad_t);
    if (ci >= L.cin || k >= L.taps * L.ys) return 0.f;
    const int t = k / L.ys, co = k - t * L.ys;
    const bool real = ci >= L.c1s || ci < L.c1;
    if (co >= L.cout || !real) return 0.f;
    const int cir = ci < L.c1s ? ci : L.c1 + (ci - L.c1s);
    return w[((int64_t)co * L.taps + (L.taps - 1 - t)) * L.cin_real + cir];
}

// The transposed copy is written in tiles of 16 input channels x 64 k
// entries through LDS: the master weights are read along the input channels
// (16 consecutive floats per k entry) and wt is written along k (8 bytes per
// lane, 128 bytes per channel row), instead of one gather per element at the
// stride of a whole output channel.
constexpr int kWtTileCi = 16, kWtTileK = 64;

// Every layer's packed and transposed weights in one launch.  Segment 2l is
// layer l's wp (8 elements per thread), segment 2l + 1 its wt (one tile per
// block); each block serves one segment (the first whose cumulative block
// count exceeds blockIdx.x), so the table is read with block-uniform indices.
__global__ void __launch_bounds__(256) k_pack_all(PackTable t, const float* __restrict__ theta) {
    __shared__ float tile[kWtTileK][kWtTileCi + 1];
    int seg = 0;
    while ((int64_t)blockIdx.x >= t.blk[seg]) ++seg;
    const int64_t first = seg ? t.blk[seg - 1] : 0;
    const int64_t b = (int64_t)blockIdx.x - first;
    const PackLayer& L = t.l[seg >> 1];
    const float* w = theta + L.woff;
    if (!(seg & 1)) {
        // 8 consecutive k entries per thread (one tap: cin is a multiple of 8), 16 bytes
        const int64_t i = (b * 256 + threadIdx.x) * 8;
        if (i >= (int64_t)L.coutp * L.kpad) return;
        bf16x8 o;
#pragma unroll
        for (int u = 0; u < 8; ++u) o[u] = (__bf16)pack_w_elem(L, i + u, w);
        *(bf16x8*)(L.wp + i) = o;
        return;
    }
    const int nkt = (L.kpad_t + kWtTileK - 1) / kWtTileK;
    const int ci0 = (int)(b / nkt) * kWtTileCi, k0 = (int)(b % nkt) * kWtTileK;
    {
        // 4 lanes per k entry, 4 consecutive input channels each
        const int kk = threadIdx.x >> 2, c4 = (threadIdx.x & 3) * 4;
        const int k = k0 + kk;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            tile[kk][c4 + u] = k < L.kpad_t ? pack_wt_elem(L, (int64_t)(ci0 + c4 + u) * L.kpad_t + k, w)
                                            : 0.f;
    }
    __syncthreads();
    // 16 lanes per input channel, 4 consecutive k entries (8 bytes) each
    const int cl = threadIdx.x >> 4, k4 = (threadIdx.x & 15) * 4;
    if (k0 + k4 >= L.kpad_t) return;  // kpad_t is a multiple of 4: whole groups
    bf16x4 o;
#pragma unroll
    for (int u = 0; u < 4; ++u) o[u] = (__bf16)tile[k4 + u][cl];
    *(bf16x4*)(L.wt + (int64_t)(ci0 + cl) * L.kpad_t + k0 + k4) = o;
}

__device__ __forceinline__ int64_t fine_index(int s, int z, int y, int x, int lg) {
    return ((int64_t)s << (3 * lg)) + ((int64_t)z << (2 * lg)) + ((int64_t)y << lg) + x;
}

// thread per (coarse cell, group of 8 channels)
__global__ void k_pool(int n, int lg, int c, const __bf16* __restrict__ x, __bf16* __restrict__ y) {
    const int h = lg - 1, cg = c / 8;
    const int64_t Vc = (int64_t)1 << (3 * h);
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * Vc * cg) return;
    const int g = (int)(idx % cg);
    const int64_t vc = idx / cg;
    const int s = (int)(vc >> (3 * h));
    const int rem = (int)(vc & (Vc - 1));
    const int Z = rem >> (2 * h), Y = (rem >> h) & ((1 << h) - 1), X = rem & ((1 << h) - 1);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int64_t vf = fine_index(s, 2 * Z + dz, 2 * Y + dy, 2 * X + dx, lg);
                const bf16x8 t = *(const bf16x8*)(x + vf * c + g * 8);
#pragma unroll
                for (int i = 0; i < 8; ++i) acc[i] += (float)t[i];
            }
    bf16x8 o;
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = (__bf16)(acc[i] * 0.125f);
    *(bf16x8*)(y + vc * c + g * 8) = o;
}

// thread per (fine cell, group of 8 channels)
__global__ void k_pool_bwd_add(int n, int lg, int c, const __bf16* __restrict__ dy,
                               const __bf16* __restrict__ skip, int ctot,
                               const __bf16* __restrict__ ymask, __bf16* __restrict__ dx) {
    const int h = lg - 1, cg = c / 8, G = 1 << lg;
    const int64_t V = (int64_t)1 << (3 * lg);
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * V * cg) return;
    const int g = (int)(idx % cg);
    const int64_t v = idx / cg;
    const int s = (int)(v >> (3 * lg));
    const int rem = (int)(v & (V - 1));
    const int z = rem >> (2 * lg), y = (rem >> lg) & (G - 1), x = rem & (G - 1);
    const int64_t vc = ((int64_t)s << (3 * h)) + ((int64_t)(z >> 1) << (2 * h)) +
                       ((int64_t)(y >> 1) << h) + (x >> 1);
    const bf16x8 p = *(const bf16x8*)(dy + vc * c + g * 8);
    bf16x8 o;
    if (skip) {
        const bf16x8 k = *(const bf16x8*)(skip + v * ctot + g * 8);
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = (__bf16)((float)p[i] * 0.125f + (float)k[i]);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = (__bf16)((float)p[i] * 0.125f);
    }
    if (ymask) {
        const bf16x8 mk = *(const bf16x8*)(ymask + v * c + g * 8);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!((float)mk[i] > 0.f)) o[i] = (__bf16)0.f;
    }
    *(bf16x8*)(dx + v * c + g * 8) = o;
}

// thread per (coarse cell, group of 8 channels)
__global__ void k_up_bwd(int n, int lg, int c, const __bf16* __restrict__ dcat, int ctot, int coff,
                         const __bf16* __restrict__ ymask, __bf16* __restrict__ dlow) {
    const int h = lg - 1, cg = c / 8;
    const int64_t Vc = (int64_t)1 << (3 * h);
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * Vc * cg) return;
    const int g = (int)(idx % cg);
    const int64_t vc = idx / cg;
    const int s = (int)(vc >> (3 * h));
    const int rem = (int)(vc & (Vc - 1));
    const int Z = rem >> (2 * h), Y = (rem >> h) & ((1 << h) - 1), X = rem & ((1 << h) - 1);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int64_t vf = fine_index(s, 2 * Z + dz, 2 * Y + dy, 2 * X + dx, lg);
                const bf16x8 t = *(const bf16x8*)(dcat + vf * ctot + coff + g * 8);
#pragma unroll
                for (int i = 0; i < 8; ++i) acc[i] += (float)t[i];
            }
    bf16x8 o;
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = (__bf16)acc[i];
    if (ymask) {
        const bf16x8 mk = *(const bf16x8*)(ymask + vc * c + g * 8);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!((float)mk[i] > 0.f)) o[i] = (__bf16)0.f;
    }
    *(bf16x8*)(dlow + vc * c + g * 8) = o;
}

__global__ void k_inputs(int n, int lg, SampleFloats lra, __bf16* __restrict__ x) {
    const int G = 1 << lg;
    const int64_t V = (int64_t)1 << (3 * lg);
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (int64_t)n * V) return;
    const int s = (int)(v >> (3 * lg));
    const int rem = (int)(v & (V - 1));
    const int z = rem >> (2 * lg), y = (rem >> lg) & (G - 1), xx = rem & (G - 1);
    const float inv = 2.0f / (float)G;
    bf16x8 o;
    o[0] = (__bf16)((lra.v[s] - 4.0f) * 0.5f);
    o[1] = (__bf16)((xx + 0.5f) * inv - 1.0f);
    o[2] = (__bf16)((y + 0.5f) * inv - 1.0f);
    o[3] = (__bf16)((z + 0.5f) * inv - 1.0f);
    o[4] = o[5] = o[6] = o[7] = (__bf16)0.f;
    *(bf16x8*)(x + v * 8) = o;
}

// The 1 x 1 x 1 head on the vector units (it reads 32 bytes and writes 16
// per voxel, far too little work for the matrix cores): kHeadIn BF16
// channels-last inputs -> kHeadOut FP32 outputs, channel-first, with the
// FP32 master weights w[co][ci] and bias b[co].  One thread per voxel.
constexpr int kHeadIn = 16, kHeadOut = 4, kHeadGrad = kHeadOut * kHeadIn + kHeadOut;

__device__ __forceinline__ void load_head_input(const __bf16* __restrict__ x, int64_t v,
                                                float* xf) {
    const bf16x8 lo = *(const bf16x8*)(x + v * kHeadIn);
    const bf16x8 hi = *(const bf16x8*)(x + v * kHeadIn + 8);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        xf[i] = (float)lo[i];
        xf[8 + i] = (float)hi[i];
    }
}

__global__ void __launch_bounds__(256) k_head_forward(int n, int lg, const __bf16* __restrict__ x,
                                                      const float* __restrict__ w,
                                                      const float* __restrict__ b, float4 sc,
                                                      float* __restrict__ out) {
    const int64_t V = (int64_t)1 << (3 * lg);
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (int64_t)n * V) return;
    const int64_t s = v >> (3 * lg), vin = v & (V - 1);
    float xf[kHeadIn];
    load_head_input(x, v, xf);
    const float scale[kHeadOut] = {sc.x, sc.y, sc.z, sc.w};
#pragma unroll
    for (int c = 0; c < kHeadOut; ++c) {
        float acc = b[c];
#pragma unroll
        for (int i = 0; i < kHeadIn; ++i) acc = fmaf(w[c * kHeadIn + i], xf[i], acc);
        out[(s * kHeadOut + c) * V + vin] = acc * scale[c];
    }
}

// Sum over the 64 lanes of a wave with DPP lane moves (no LDS): pairs and
// quads by quad permutes, rows of 16 by rotations by 4 and 8, then row 0's
// sum into row 1 and row 2's into row 3 by the lane-15 broadcast, and row
// 1's into rows 2 and 3 by the lane-31 broadcast.  Lane 63 receives the
// total, summed in the same order every time.  Rows left out of a move add 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_moved(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}

__device__ __forceinline__ float wave_sum_in_last_lane(float v) {
    v += dpp_moved<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_moved<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_moved<0x124, 0xF>(v);  // row_ror 4
    v += dpp_moved<0x128, 0xF>(v);  // row_ror 8
    v += dpp_moved<0x142, 0xA>(v);  // row_bcast 15 (rows 1 and 3)
    v += dpp_moved<0x143, 0xC>(v);  // row_bcast 31 (rows 2 and 3)
    return v;
}

// Loss and the whole backward step of the head in one pass: per voxel the
// head's output out = b + w x (the FMA sequence of k_head_forward, so the
// same values), the output gradient d = 2 (out - t) / count (t = target
// times its scale), the
// input gradient dx[ci] = sum_co w[co][ci] d[co] (0 where the ReLU output x
// <= 0; written as BF16), and the contributions d[co] x[ci] and d[co] to the
// weight and bias gradients.  Block b takes voxels [b chunk, (b + 1) chunk);
// its sums (squared error in FP64, the kHeadGrad gradient entries in FP32)
// are added over the block in a fixed order and written to lpart[b] and
// gpart[b][kHeadGrad].
__global__ void __launch_bounds__(256) k_head_backward(
    int n, int lg, const float* __restrict__ tg, SampleInts idx, int64_t stride, float4 ts,
    const __bf16* __restrict__ x, const float* __restrict__ w, const float* __restrict__ b,
    int64_t chunk, __bf16* __restrict__ dx, double* __restrict__ lpart,
    float* __restrict__ gpart) {
    __shared__ float gred[4][kHeadGrad];
    __shared__ double lred[256];
    const int64_t V = (int64_t)1 << (3 * lg);
    const int64_t M = (int64_t)n * V;
    const float inv = (float)(2.0 / ((double)n * 4.0 * (double)V));
    const float tsc[kHeadOut] = {ts.x, ts.y, ts.z, ts.w};
    float g[kHeadGrad];
#pragma unroll
    for (int j = 0; j < kHeadGrad; ++j) g[j] = 0.f;
    double lsum = 0.0;
    const int64_t v0 = (int64_t)blockIdx.x * chunk;
    const int64_t v1 = v0 + chunk < M ? v0 + chunk : M;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
        const int s = (int)(v >> (3 * lg));
        const int64_t vin = v & (V - 1);
        float xf[kHeadIn];
        load_head_input(x, v, xf);
        float d[kHeadOut];
#pragma unroll
        for (int c = 0; c < kHeadOut; ++c) {
            float ov = b[c];
#pragma unroll
            for (int i = 0; i < kHeadIn; ++i) ov = fmaf(w[c * kHeadIn + i], xf[i], ov);
            const float tv = tg[(int64_t)idx.v[s] * stride + c * V + vin] * tsc[c];
            const double e = (double)ov - (double)tv;
            lsum += e * e;
            d[c] = (float)e * inv;
        }
        bf16x8 lo, hi;
#pragma unroll
        for (int i = 0; i < kHeadIn; ++i) {
            float acc = 0.f;
#pragma unroll
            for (int c = 0; c < kHeadOut; ++c) acc = fmaf(w[c * kHeadIn + i], d[c], acc);
            const __bf16 r = (__bf16)(xf[i] > 0.f ? acc : 0.f);
            if (i < 8)
                lo[i] = r;
            else
                hi[i - 8] = r;
        }
        *(bf16x8*)(dx + v * kHeadIn) = lo;
        *(bf16x8*)(dx + v * kHeadIn + 8) = hi;
#pragma unroll
        for (int c = 0; c < kHeadOut; ++c) {
#pragma unroll
            for (int i = 0; i < kHeadIn; ++i) g[c * kHeadIn + i] = fmaf(d[c], xf[i], g[c * kHeadIn + i]);
            g[kHeadOut * kHeadIn + c] += d[c];
        }
    }
    // the wave's 64 lanes by DPP moves, then the 4 waves in order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kHeadGrad; ++j) {
        const float val = wave_sum_in_last_lane(g[j]);
        if (lane == 63) gred[wave][j] = val;
    }
    lred[threadIdx.x] = lsum;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) lred[threadIdx.x] += lred[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x < kHeadGrad)
        gpart[(int64_t)blockIdx.x * kHeadGrad + threadIdx.x] =
            ((gred[0][threadIdx.x] + gred[1][threadIdx.x]) + gred[2][threadIdx.x]) +
            gred[3][threadIdx.x];
    if (threadIdx.x == 0) lpart[blockIdx.x] = lred[0];
}

// The head's block sums in one launch.  Blocks j < width: out[j] = sum over
// rows r of in[r][j] (rows x width, FP32); the last block: loss = sum of the
// rows FP64 partials lp.  Thread t adds rows t, t + 256, ... in order, then a
// fixed tree adds the 256 thread sums.
template <typename T>
__device__ __forceinline__ T block_tree_sum(T* red, T v) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    return red[0];
}

__global__ void __launch_bounds__(256) k_head_sums(const float* __restrict__ in, int rows,
                                                   int width, float* __restrict__ out,
                                                   const double* __restrict__ lp,
                                                   double* __restrict__ loss) {
    __shared__ float redf[256];
    __shared__ double redd[256];
    const int j = blockIdx.x;
    if (j < width) {
        float acc = 0.f;
        for (int r = threadIdx.x; r < rows; r += 256) acc += in[(int64_t)r * width + j];
        const float t = block_tree_sum(redf, acc);
        if (threadIdx.x == 0) out[j] = t;
    } else {
        double acc = 0.0;
        for (int r = threadIdx.x; r < rows; r += 256) acc += lp[r];
        const double t = block_tree_sum(redd, acc);
        if (threadIdx.x == 0) loss[0] = t;
    }
}

__global__ void k_adam(int64_t count, float* __restrict__ th, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ g, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_zero(float* __restrict__ p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.f;
}

__global__ void k_bf16_to_f32(const __bf16* __restrict__ x, int64_t cells, int cs, int c,
                              float* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cells * c) return;
    const int64_t v = i / c;
    const int ch = (int)(i - v * c);
    y[i] = (float)x[v * cs + ch];
}

__global__ void k_cf_to_cl(const float* __restrict__ x, int n, int64_t V, int c,
                           float* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * V * c) return;
    const int ch = (int)(i % c);
    const int64_t v = (i / c) % V;
    const int64_t s = i / (c * V);
    y[i] = x[(s * c + ch) * V + v];
}

// Forward / input-gradient convolution on LDS-staged bricks (3x3x3 taps,
// BF16 output, grids of at least 16 cells, input channels a multiple of 16,
// or 8 with no second tensor).  A block of 8 waves computes 16 x 4 x 8 output
// voxels (wave w the plane z0 + w, its four 16-voxel row tiles y0 .. y0 + 3)
// for NSUB * 16 output channels.  Per 16 input channels the block copies the
// 18 x 6 x 10 input halo (channels-last, 32 bytes per voxel: lane r reads
// voxel r and its second 8 channels sit 16 bytes on, which the LDS serves
// without bank conflicts) and the chunk's weights into LDS with direct-to-LDS
// buffer loads (no register staging, every load of the chunk in flight at
// once), so every A fragment (8 channels of one voxel for one tap) is one LDS
// read.  A k step of 32 takes two taps of the 16 channels, paired so that
// the second lies a fixed displacement from the first within each group of
// steps (two planes on, two rows on, two voxels on, or a slot of zero
// weights): a lane's LDS addresses are then a base register per group plus
// a compile-time offset, with no per-step index arithmetic.
constexpr int kCvVox = 16;                  // LDS elements per voxel
constexpr int kCvPlanes = 8;                // output planes (waves) per block
constexpr int kCvHalo = 18 * 6 * (kCvPlanes + 2);  // halo voxels
constexpr int kCvHaloItems = 2 * kCvHalo;   // 16-byte halo items of a chunk
constexpr int kCvHaloBuf = kCvHaloItems + 16;  // + the tail of the last partial wave
constexpr int kCvSlots = 28;                // 27 taps + a zero-weight slot
constexpr int kCvWItemsRow = 2 * kCvSlots + 2;  // 16-byte weight items per row (+ 32 B pad)
constexpr int kCvWRow = 8 * kCvWItemsRow;   // elements per LDS weight row (928 B, 32 mod 64)

// Step p (0..13) of the k loop takes tap p in lanes q < 2 and tap
// cv_pair_tap(p) in lanes q >= 2 (-1: the zero slot); cv_pair_shift(p) is
// the second tap's halo position minus the first's, in voxels.
__device__ constexpr int cv_pair_tap(int p) {
    return p <= 8 ? p + 18 : p <= 11 ? p + 6 : p == 12 ? 14 : -1;
}
__device__ constexpr int cv_pair_shift(int p) {
    return p <= 8 ? 2 * 108 : p <= 11 ? 2 * 18 : p == 12 ? 2 : 0;
}
// halo position of tap t = (dz + 1) * 9 + (dy + 1) * 3 + dx + 1, relative to
// the output voxel's (-1, -1, -1) neighbour
__device__ constexpr int cv_tap_offset(int t) { return (t / 9) * 108 + ((t / 3) % 3) * 18 + t % 3; }

template <int NSUB>
__global__ void __launch_bounds__(64 * kCvPlanes)
    __attribute__((amdgpu_waves_per_eu(NSUB == 1 ? 6 : 4))) k_conv_brick(ConvArgs a) {
    constexpr int kThreads = 64 * kCvPlanes;
    constexpr int kWItems = NSUB * 16 * kCvWItemsRow;
    constexpr int kWBuf = (kWItems + 63) / 64 * 64;  // whole waves of 16-byte items
    __shared__ __attribute__((aligned(16))) __bf16 xs[kCvHaloBuf * 8];
    __shared__ __attribute__((aligned(16))) __bf16 wl[kWBuf * 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4, hi = q >> 1;
    const int lg = a.lg, G = 1 << lg;
    const int nbx = G >> 4, nby = G >> 2, nbz = G / kCvPlanes;
    // blocks i, i + 8, ... run on one XCD (dispatch is round-robin over the
    // eight): give each XCD a contiguous range of bricks, whose halos overlap
    // in its L2 (the grid's x size is a multiple of 8 for G >= 16)
    int64_t bid = (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const int x0 = (int)(bid % nbx) * 16;
    bid /= nbx;
    const int y0 = (int)(bid % nby) * 4;
    bid /= nby;
    const int z0 = (int)(bid % nbz) * kCvPlanes;
    const int smp = (int)(bid / nbz);
    const int cobase = blockIdx.y * NSUB * 16;
    floatx4 acc[4][NSUB];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NSUB; ++j) acc[m][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int ch = (q & 1) * 8;
    // LDS byte addresses of this lane: A (halo) per shift group, B (weights)
    const uint32_t lb = (uint32_t)(wave * 108 + r);
    const uint32_t vA0 = ((lb + hi * 2 * 108) * kCvVox + ch) * 2;
    const uint32_t vA1 = ((lb + hi * 2 * 18) * kCvVox + ch) * 2;
    const uint32_t vA2 = ((lb + hi * 2) * kCvVox + ch) * 2;
    const uint32_t vA3 = (lb * kCvVox + ch) * 2;
    const uint32_t vB = (uint32_t)(r * kCvWRow + hi * 16 + ch) * 2;
    const char* xsb = (const char*)xs;
    const char* wlb = (const char*)wl;
    // Loads go through range-checked buffer resources: a position outside
    // the grid (or the tensor, or a weight item of the zero slot or padding)
    // reads past the end and lands as zeros.
    const int h = lg - 1;
    for (int c0 = 0; c0 < a.cin; c0 += 16) {
        const bool lo = c0 < a.c1s;  // x1's channels, else x2's (c1s is then a multiple of 16)
        const int chans = lo ? a.c1s : a.c2;
        const int hl = lo ? lg : h;  // the tensor's grid: 2^hl cells a side
        const int sh = lo ? 0 : 1;   // coarse tensor: the fine cell's parent
        const int64_t vs = (int64_t)1 << (3 * hl);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<__bf16*>((lo ? a.x1 : a.x2) + (int64_t)smp * vs * chans), (short)0,
            (int)(uint32_t)(vs * chans * 2), 0x00020000);
        const int cloc = lo ? c0 : c0 - a.c1s;
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        // halo item t (voxel t / 2, channel half t % 2) lands at LDS byte 16 t
#pragma unroll
        for (int i = 0; i < (kCvHaloItems + kThreads - 1) / kThreads; ++i) {
            const int tb = i * kThreads + wv * 64;
            if (tb >= kCvHaloItems) continue;
            const int t = tb + lane;
            const int half = t & 1, hv = t >> 1;
            const int hx = hv % 18, hy = (hv / 18) % 6, hz = hv / 108;
            const int xx = x0 + hx - 1, yy = y0 + hy - 1, zz = z0 + hz - 1;
            const bool ok = t < kCvHaloItems && c0 + half * 8 < a.cin && (unsigned)xx < (unsigned)G &&
                            (unsigned)yy < (unsigned)G && (unsigned)zz < (unsigned)G;
            const uint32_t vox = ((uint32_t)(zz >> sh) << (2 * hl)) + ((uint32_t)(yy >> sh) << hl) +
                                 (uint32_t)(xx >> sh);
            const uint32_t off = ((vox * (uint32_t)chans + (uint32_t)(cloc + half * 8)) * 2u) |
                                 ((uint32_t)!ok << 31);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_ptr)&xs[tb * 8], 16, off, 0, 0, 0);
        }
        const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<__bf16*>(a.w), (short)0, (int)(uint32_t)((int64_t)a.wrows * a.kpad * 2),
            0x00020000);
        // weight item t: row t / 58 (output channel cobase + row), slot s =
        // (t % 58) / 2 (tap s / 2 for even s, the paired tap for odd s), 8
        // channels of half t % 2; items 56, 57 of a row are padding.  (With 8
        // input channels the upper half holds the next tap's weights, which
        // meet zero inputs, and stays inside the row since 27 * 8 + 8 <= kpad.)
#pragma unroll
        for (int i = 0; i < (kWBuf + kThreads - 1) / kThreads; ++i) {
            const int tb = i * kThreads + wv * 64;
            if (tb >= kWBuf) continue;
            const int t = tb + lane;
            const int row = t / kCvWItemsRow, rem = t - row * kCvWItemsRow;
            const int slot = rem >> 1, half = rem & 1, p = slot >> 1;
            const int tap = (slot & 1) ? cv_pair_tap(p) : p;
            const bool ok = t < kWItems && rem < 2 * kCvSlots && tap >= 0 && cobase + row < a.wrows;
            const uint32_t off =
                ((uint32_t)((cobase + row) * a.kpad + tap * a.cin + c0 + half * 8) * 2u) |
                ((uint32_t)!ok << 31);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (lds_void_ptr)&wl[tb * 8], 16, off, 0, 0, 0);
        }
        // this wave's copies have landed (vmcnt 0; expcnt and lgkmcnt left at their maxima)
        __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 14; ++p) {
            const int d = cv_pair_shift(p);
            const uint32_t va = d == 2 * 108 ? vA0 : d == 2 * 18 ? vA1 : d == 2 ? vA2 : vA3;
            const int toff = cv_tap_offset(p);
            bf16x8 bv[NSUB], av[4];
#pragma unroll
            for (int j = 0; j < NSUB; ++j)
                bv[j] = *(const bf16x8*)(wlb + vB + (j * 16 * kCvWRow + p * 32) * 2);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                av[m] = *(const bf16x8*)(xsb + va + (toff + m * 18) * kCvVox * 2);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int j = 0; j < NSUB; ++j)
                    acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[j], acc[m][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // D rows 4q .. 4q+3 are x offsets, column r an output channel
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int64_t vrow = ((((int64_t)smp << lg) + z0 + wave) << (2 * lg)) +
                             ((int64_t)(y0 + m) << lg) + x0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t vo = vrow + q * 4 + i;
#pragma unroll
            for (int j = 0; j < NSUB; ++j) {
                const int co = cobase + j * 16 + r;
                if (co < a.ys) {
                    float val = 0.f;
                    if (co < a.cout) {
                        val = acc[m][j][i] + (a.bias ? a.bias[co] : 0.f);
                        if (a.relu) val = fmaxf(val, 0.f);
                        if (a.omask && !((float)a.omask[vo * a.ys + co] > 0.f)) val = 0.f;
                    }
                    a.out[vo * a.ys + co] = (__bf16)val;
                }
            }
        }
    }
}

// Forward / input-gradient convolution on grids of 8 cells (3x3x3 taps,
// input channels a multiple of 16, one input tensor), split over the input
// channel groups: a block of 8 waves computes one sample's 8 x 8 x 8 outputs
// (wave w the plane z = w: four 16-voxel tiles of two 8-cell rows) for 16
// output channels from one 16-channel input group and writes FP32 partial
// sums, which k_conv_small_sum adds in a fixed order (with the bias, ReLU and
// mask).  Split this way a 128-channel layer of batch 8 has 512 blocks
// instead of 64.  The 10 x 10 x 10 halo (channels-last, 32 bytes a voxel)
// and the group's weights (in the brick convolution's tap-pair order) are
// copied with direct-to-LDS loads; the pairs' displacements are two planes
// (200 voxels), two rows (20) or two voxels.
constexpr int kSmHaloItems = 2 * 1000;   // 16-byte halo items
constexpr int kSmHaloBuf = 32 * 64;      // whole waves of items

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6)))
k_conv_small(ConvArgs a, float* __restrict__ part) {
    constexpr int kThreads = 512;
    constexpr int kWItems = 16 * kCvWItemsRow;
    constexpr int kWBuf = (kWItems + 63) / 64 * 64;
    __shared__ __attribute__((aligned(16))) __bf16 xs[kSmHaloBuf * 8];
    __shared__ __attribute__((aligned(16))) __bf16 wl[kWBuf * 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4, hi = q >> 1;
    const int nch = a.cin / 16;
    const int smp = blockIdx.x / nch, chunk = blockIdx.x % nch;
    const int c0 = chunk * 16;
    const int cobase = blockIdx.y * 16;
    const int ch = (q & 1) * 8;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // halo item t (voxel t / 2 of 10 x 10 x 10, channel half t % 2) -> LDS byte 16 t;
    // positions outside the grid, channel halves past cin and the padding items read zeros
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<__bf16*>(a.x1 + (int64_t)smp * 512 * a.c1s), (short)0, 512 * a.c1s * 2,
        0x00020000);
#pragma unroll
    for (int i = 0; i < kSmHaloBuf / kThreads; ++i) {
        const int tb = i * kThreads + wv * 64;
        const int t = tb + lane;
        const int half = t & 1, hv = t >> 1;
        const int xx = hv % 10 - 1, yy = (hv / 10) % 10 - 1, zz = hv / 100 - 1;
        const bool ok = t < kSmHaloItems && c0 + half * 8 < a.cin && (unsigned)xx < 8u &&
                        (unsigned)yy < 8u && (unsigned)zz < 8u;
        const uint32_t vox = ((uint32_t)zz << 6) + ((uint32_t)yy << 3) + (uint32_t)xx;
        const uint32_t off = ((vox * (uint32_t)a.c1s + (uint32_t)(c0 + half * 8)) * 2u) |
                             ((uint32_t)!ok << 31);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_ptr)&xs[tb * 8], 16, off, 0, 0, 0);
    }
    // weight item t: row t / 58 (output channel cobase + row), tap-pair slot
    // (t % 58) / 2, channel half t % 2; items 56, 57 of a row pad
    const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<__bf16*>(a.w), (short)0, (int)(uint32_t)((int64_t)a.wrows * a.kpad * 2), 0x00020000);
#pragma unroll
    for (int i = 0; i < (kWBuf + kThreads - 1) / kThreads; ++i) {
        const int tb = i * kThreads + wv * 64;
        if (tb >= kWBuf) continue;
        const int t = tb + lane;
        const int row = t / kCvWItemsRow, rem = t - row * kCvWItemsRow;
        const int slot = rem >> 1, half = rem & 1, p = slot >> 1;
        const int tap = (slot & 1) ? cv_pair_tap(p) : p;
        const bool ok = t < kWItems && rem < 2 * kCvSlots && tap >= 0 && cobase + row < a.wrows;
        const uint32_t off =
            ((uint32_t)((cobase + row) * a.kpad + tap * a.cin + c0 + half * 8) * 2u) |
            ((uint32_t)!ok << 31);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (lds_void_ptr)&wl[tb * 8], 16, off, 0, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));  // vmcnt 0: this wave's copies landed
    __syncthreads();
    // lane r of tile m is the output voxel (z = w, y = 2 m + r / 8, x = r % 8)
    const uint32_t lb = (uint32_t)(wave * 100 + (r >> 3) * 10 + (r & 7));
    const uint32_t vA0 = ((lb + hi * 200) * kCvVox + ch) * 2;
    const uint32_t vA1 = ((lb + hi * 20) * kCvVox + ch) * 2;
    const uint32_t vA2 = ((lb + hi * 2) * kCvVox + ch) * 2;
    const uint32_t vA3 = (lb * kCvVox + ch) * 2;
    const uint32_t vB = (uint32_t)(r * kCvWRow + hi * 16 + ch) * 2;
    const char* xsb = (const char*)xs;
    const char* wlb = (const char*)wl;
    floatx4 acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 14; ++p) {
        const uint32_t va = p <= 8 ? vA0 : p <= 11 ? vA1 : p == 12 ? vA2 : vA3;
        const int toff = (p / 9) * 100 + ((p / 3) % 3) * 10 + p % 3;  // halo position of tap p
        const bf16x8 bv = *(const bf16x8*)(wlb + vB + p * 64);
        bf16x8 av[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) av[m] = *(const bf16x8*)(xsb + va + (toff + m * 20) * kCvVox * 2);
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv, acc[m], 0, 0, 0);
    }
    // D rows 4q .. 4q+3 of tile m are voxels 16 m + 4 q + i of the plane, column r a channel
    const int Cp = gridDim.y * 16;
    float* pp = part + ((int64_t)chunk * a.n + smp) * 512 * Cp;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            pp[(int64_t)(wave * 64 + 16 * m + 4 * q + i) * Cp + cobase + r] = acc[m][i];
}

// out[v][co] = (ReLU)(bias + sum over the nch input groups of the partials,
// in group order), 0 where omask <= 0 and for co >= cout; one thread per output.
__global__ void k_conv_small_sum(const float* __restrict__ part, int nch, int64_t cells, int Cp,
                                 const float* __restrict__ bias, int relu,
                                 const __bf16* __restrict__ omask, int cout, int ys,
                                 __bf16* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cells * ys) return;
    const int64_t v = i / ys;
    const int co = (int)(i - v * ys);
    float val = 0.f;
    if (co < cout) {
        float sum = 0.f;
        for (int c = 0; c < nch; ++c) sum += part[((int64_t)c * cells + v) * Cp + co];
        val = sum + (bias ? bias[co] : 0.f);
        if (relu) val = fmaxf(val, 0.f);
        if (omask && !((float)omask[i] > 0.f)) val = 0.f;
    }
    out[i] = (__bf16)val;
}

// Partial-sum floats k_conv_small needs for the convolution a describes
// (coutp output rows), or 0 if it does not apply.
int64_t conv_small_floats(const ConvArgs& a, int coutp) {
    if (a.lg != 3 || a.taps != 27 || a.c2 != 0 || a.cin % 16 != 0 || a.kpad < 27 * a.cin)
        return 0;
    return (int64_t)(a.cin / 16) * a.n * 512 * coutp;
}

template <int MT, int KS>
hipError_t launch_conv_mt(const ConvArgs& a, int coutp, hipStream_t s) {
    const int64_t M = (int64_t)a.n << (3 * a.lg);
    const int sub = coutp / 16;
    const int nsub = sub % 4 == 0 ? 4 : sub % 3 == 0 ? 3 : sub % 2 == 0 ? 2 : 1;
    const dim3 grid(ceil_div(M, 16 * MT), sub / nsub), block(64 * KS);
    switch (nsub) {
        case 4: hipLaunchKernelGGL((k_conv<4, MT, KS>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_conv<3, MT, KS>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_conv<2, MT, KS>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((k_conv<1, MT, KS>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

// Four voxel tiles per wave when that still leaves at least 2048 blocks (so
// each weight fragment serves 64 voxels).  Otherwise one tile, and the k
// range is split over 2 or 4 waves per block when there are fewer than
// 4096 or 1024 blocks and at least two steps of 32 per wave (8 waves were
// measured no faster on the 8^3 layers).
hipError_t launch_conv(const ConvArgs& a, int coutp, float* scratch, int64_t scratch_floats,
                       hipStream_t s) {
    const int64_t M = (int64_t)a.n << (3 * a.lg);
    const int sub = coutp / 16;
    const int64_t small = conv_small_floats(a, coutp);
    if (small > 0 && scratch && small <= scratch_floats) {
        // grids of 8 cells: split over the input channel groups, then summed
        ConvArgs b = a;
        b.wrows = coutp;
        hipLaunchKernelGGL(k_conv_small, dim3(a.n * (a.cin / 16), sub), dim3(512), 0, s, b, scratch);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t outs = M * a.ys;
        hipLaunchKernelGGL(k_conv_small_sum, dim3((unsigned)ceil_div(outs, 256)), dim3(256), 0, s,
                           scratch, a.cin / 16, M, coutp, a.bias, a.relu, a.omask, a.cout, a.ys,
                           a.out);
        return hipGetLastError();
    }
    const int nsub = sub % 4 == 0 ? 4 : sub % 3 == 0 ? 3 : sub % 2 == 0 ? 2 : 1;
    // (8 input channels, the first layer, take a 16-channel group whose upper
    // half reads zeros; its weight rows there hold the next tap's weights,
    // which multiply those zeros, and stay inside the row since 27 * 8 + 8 <=
    // kpad.)
    if (a.taps == 27 && a.lg >= 4 && a.kpad >= 27 * a.cin &&
        (a.cin % 16 == 0 || (a.cin == 8 && a.c2 == 0)) && (a.c2 == 0 || a.c1s % 16 == 0)) {
        // one output-channel group per block (more blocks, fewer registers),
        // except for 3 groups of 16 on grids of 32 and more, where one block
        // serving all three was faster (measured: 48 channels on 64^3 243
        // against 257 us, 96 on 32^3 75 against 98 us; 32 channels 40 -> 36 us)
        const int64_t G = (int64_t)1 << a.lg;
        const int nb = a.lg >= 5 && nsub == 3 ? 3 : 1;
        const dim3 grid((unsigned)((G / 16) * (G / 4) * (G / kCvPlanes) * a.n), sub / nb);
        const dim3 block(64 * kCvPlanes);
        ConvArgs b = a;
        b.wrows = coutp;
        if (nb == 3)
            hipLaunchKernelGGL(k_conv_brick<3>, grid, block, 0, s, b);
        else
            hipLaunchKernelGGL(k_conv_brick<1>, grid, block, 0, s, b);
        return hipGetLastError();
    }
    const int64_t waves4 = (int64_t)ceil_div(M, 64) * (sub / nsub);
    if (waves4 >= 2048) return launch_conv_mt<4, 1>(a, coutp, s);
    const int64_t waves1 = (int64_t)ceil_div(M, 16) * (sub / nsub);
    const int ksteps = a.kpad / 32;
    if (waves1 < 1024 && ksteps >= 8) return launch_conv_mt<1, 4>(a, coutp, s);
    if (waves1 < 4096 && ksteps >= 4) return launch_conv_mt<1, 2>(a, coutp, s);
    return launch_conv_mt<1, 1>(a, coutp, s);
}

}  // namespace

ConvGeom make_geom(int n, int lg, int taps, int c1, int c2, int cout) {
    ConvGeom g;
    g.n = n;
    g.lg = lg;
    g.taps = taps;
    g.c1 = c1;
    g.c1s = round_up(c1, 8);
    g.c2 = c2;
    g.cin = g.c1s + c2;
    g.K = taps * g.cin;
    g.kpad = round_up(g.K, 32);
    g.cout = cout;
    g.coutp = round_up(cout, 16);
    g.ys = round_up(cout, 8);
    g.kpad_t = round_up(taps * g.ys, 32);
    g.cinp = round_up(g.cin, 16);
    return g;
}

hipError_t pack_weights(int layers, const ConvGeom* g, const float* theta, const int64_t* woff,
                        __bf16* const* wp, __bf16* const* wt, hipStream_t s) {
    if (layers < 1 || layers > kMaxPackLayers) return hipErrorInvalidValue;
    PackTable t;
    int64_t blocks = 0;
    for (int l = 0; l < kMaxPackLayers; ++l) {
        PackLayer& L = t.l[l];
        if (l >= layers) {
            L = PackLayer{};
            t.blk[2 * l] = t.blk[2 * l + 1] = blocks;
            continue;
        }
        L.wp = wp[l];
        L.wt = wt[l];
        L.woff = woff[l];
        L.coutp = g[l].coutp;
        L.kpad = g[l].kpad;
        L.cout = g[l].cout;
        L.K = g[l].K;
        L.cin = g[l].cin;
        L.c1 = g[l].c1;
        L.c1s = g[l].c1s;
        L.taps = g[l].taps;
        L.cin_real = g[l].c1 + g[l].c2;
        L.cinp = g[l].cinp;
        L.kpad_t = g[l].kpad_t;
        L.ys = g[l].ys;
        blocks += ceil_div((int64_t)L.coutp * L.kpad, 256 * 8);
        t.blk[2 * l] = blocks;
        // (kpad is a multiple of 8, cinp of kWtTileCi, kpad_t of 4)
        if (L.kpad % 8 || L.cinp % kWtTileCi || L.kpad_t % 4) return hipErrorInvalidValue;
        blocks += (int64_t)(L.cinp / kWtTileCi) * ceil_div((int64_t)L.kpad_t, kWtTileK);
        t.blk[2 * l + 1] = blocks;
    }
    hipLaunchKernelGGL(k_pack_all, dim3((unsigned)blocks), dim3(256), 0, s, t, theta);
    return hipGetLastError();
}

hipError_t conv_forward(const ConvGeom& g, const __bf16* x1, const __bf16* x2, const __bf16* wp,
                        const float* bias, int relu, __bf16* out, float* scratch,
                        int64_t scratch_floats, hipStream_t s) {
    if (!x1 || !wp || !out || (g.c2 > 0 && (!x2 || g.lg < 1)) || g.c1s % 8 || g.c2 % 8)
        return hipErrorInvalidValue;
    ConvArgs a;
    a.x1 = x1;
    a.x2 = x2;
    a.w = wp;
    a.bias = bias;
    a.out = out;
    a.omask = nullptr;
    a.n = g.n;
    a.lg = g.lg;
    a.taps = g.taps;
    a.c1s = g.c1s;
    a.c2 = g.c2;
    a.cin = g.cin;
    a.K = g.K;
    a.kpad = g.kpad;
    a.cout = g.cout;
    a.ys = g.ys;
    a.relu = relu;
    return launch_conv(a, g.coutp, scratch, scratch_floats, s);
}

hipError_t conv_backward_data(const ConvGeom& g, const __bf16* dy, const __bf16* wt,
                              const __bf16* dxmask, __bf16* dx, float* scratch,
                              int64_t scratch_floats, hipStream_t s) {
    if (!dy || !wt || !dx) return hipErrorInvalidValue;
    ConvArgs a;
    a.x1 = dy;
    a.x2 = nullptr;
    a.w = wt;
    a.bias = nullptr;
    a.out = dx;
    a.omask = dxmask;
    a.n = g.n;
    a.lg = g.lg;
    a.taps = g.taps;
    a.c1s = g.ys;
    a.c2 = 0;
    a.cin = g.ys;
    a.K = g.taps * g.ys;
    a.kpad = g.kpad_t;
    a.cout = g.cin;
    a.ys = g.cin;
    a.relu = 0;
    return launch_conv(a, g.cinp, scratch, scratch_floats, s);
}

int64_t conv_scratch_floats(const ConvGeom& g) {
    ConvArgs f = {};
    f.n = g.n, f.lg = g.lg, f.taps = g.taps, f.c2 = g.c2, f.cin = g.cin, f.kpad = g.kpad;
    ConvArgs b = f;
    b.c2 = 0, b.cin = g.ys, b.kpad = g.kpad_t;
    return std::max(conv_small_floats(f, g.coutp), conv_small_floats(b, g.cinp));
}

namespace {

// Launch plan of the weight gradient: a brick kernel (grids of at least 16
// cells, 27 taps, 16/32 output channels with >= 8 input channels, 64 with
// >= 16) or the tiled kernel, its grid, and the floats of partial sums it
// writes.
struct WgradPlan {
    bool small;          // 8-cell grids: k_wgrad_small, one block per (group, sample, 32 channels)
    bool brick;
    int rs, cs;
    int chunks, groups;  // brick: channel groups x brick ranges
    int64_t per;         // brick: bricks per range
    int kt, ct, nz;      // tiled: column tiles, row tiles, voxel chunks
    int64_t vchunk;
    int64_t part_floats, bias_off;  // partial sums of every block
    int64_t rows, wwidth, bwidth;   // rows of partials, weight / bias floats per row
    int64_t scratch_floats;         // partials + the first reduction pass
    bool slices;                    // whether the first reduction pass runs
};

// Scratch of the first reduction pass, after the partials: the weight rows
// and the bias rows summed over slices of kRowSlice rows.
void finish_plan(WgradPlan* p) {
    p->slices = p->rows > 2 * kRowSlice;
    const int64_t sl = p->slices ? (p->rows + kRowSlice - 1) / kRowSlice : 0;
    p->scratch_floats = p->part_floats + sl * (p->wwidth + p->bwidth);
}

// Partial sums kept to about 32 MB and 1024 blocks: enough blocks to fill
// the chip, and a second pass that reads far less than the layer's inputs.
constexpr int64_t kPartFloats = 8 << 20;
constexpr int64_t kPartBlocks = 1024;

// Blocks of k_wgrad_tr<rs> (rs 1 or 2) for one generation on the device:
// the compute units times the blocks each holds at once, at most 2 (asked
// once per process; 512 if the runtime cannot say).  With 48-64 registers 3-4
// fit, but fewer blocks each walking more bricks were faster (64^3, batch 8:
// 16 -> 16 channels 70 -> 53 us, 32 -> 48 channels 77 -> 53 us): neighbouring
// bricks of a range share halo cells and output rows in L2.
int64_t wgrad_tr_resident(int rs) {
    static int64_t cached[2] = {0, 0};
    int64_t& c = cached[rs == 2];
    if (c == 0) {
        int dev = 0, cus = 0, per = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = rs == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_wgrad_tr<2>, 64 * kWtWaves, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_wgrad_tr<1>, 64 * kWtWaves, 0);
        c = e == hipSuccess && cus > 0 && per > 0 ? (int64_t)cus * std::min(per, 2) : 512;
    }
    return c;
}

// (The brick kernel reads the output gradient unmasked: relu != 0 takes the
// tiled kernel.)
WgradPlan wgrad_plan(const ConvGeom& g, int relu) {
    WgradPlan p = {};
    const int64_t M = (int64_t)g.n << (3 * g.lg);
    // (8 input channels, the network's first layer, takes a channel group
    // of 16 whose upper half loads zeros; only k_wgrad_tr is checked for
    // that, so 64 output channels need 16.)
    p.small = !relu && g.lg == 3 && g.taps == 27 && g.c2 == 0 && g.cin % 16 == 0 &&
              g.coutp % 32 == 0;
    if (p.small) {
        p.rs = g.coutp / 16;
        p.chunks = g.cin / 16;
        p.groups = g.n;  // partial rows: one per sample
        const int64_t blk_floats = (int64_t)27 * g.coutp * 16;
        p.bias_off = (int64_t)g.n * p.chunks * blk_floats;
        p.part_floats = p.bias_off + (int64_t)g.n * g.coutp;
        p.rows = g.n;
        p.wwidth = (int64_t)p.chunks * blk_floats;
        p.bwidth = g.coutp;
        p.slices = false;
        p.scratch_floats = p.part_floats;
        return p;
    }
    p.brick = !relu && g.lg >= 4 && g.taps == 27 &&
              (g.c2 == 0 || g.c1s % 16 == 0) &&
              ((g.cin >= 8 && (g.coutp == 16 || g.coutp == 32)) || (g.cin >= 16 && g.coutp == 64));
    if (p.brick) {
        p.rs = g.coutp / 16;
        p.chunks = ceil_div(g.cin, 16);
        // bricks of 16 x 4 x 4 voxels (k_wgrad_tr) or 16 x 4 x 2 (k_wgrad_brick)
        const int64_t nbricks = M / (p.rs == 4 ? 128 : 256);
        const int64_t blk_floats = (int64_t)27 * g.coutp * 16;
        // k_wgrad_tr: one generation of resident blocks
        const int64_t blocks = p.rs == 4 ? kPartBlocks : wgrad_tr_resident(p.rs);
        const int64_t cap = std::max<int64_t>(
            1, std::min<int64_t>(blocks, kPartFloats / blk_floats) / p.chunks);
        const int64_t groups = std::max<int64_t>(1, std::min<int64_t>(nbricks, cap));
        p.per = (nbricks + groups - 1) / groups;
        p.groups = ceil_div(nbricks, p.per);
        p.bias_off = (int64_t)p.groups * p.chunks * blk_floats;
        p.part_floats = p.bias_off + (int64_t)p.groups * g.coutp;
        p.rows = p.groups;
        p.wwidth = (int64_t)p.chunks * blk_floats;
        p.bwidth = g.coutp;
        p.slices = false;  // one pass (k_brick_partials_sum)
        p.scratch_floats = p.part_floats;
        return p;
    }
    p.rs = g.coutp >= 64 ? 4 : g.coutp >= 32 ? 2 : 1;
    p.cs = 8 / p.rs;
    p.ct = ceil_div(g.coutp, 16 * p.rs);
    p.kt = ceil_div(g.K, 16 * p.cs);
    const int64_t steps = (M + 31) / 32;
    const int64_t blk_floats = (int64_t)p.rs * 16 * p.cs * 16;
    const int64_t tiles = (int64_t)p.kt * p.ct;
    const int64_t cap = std::max<int64_t>(
        1, std::min<int64_t>(2 * kPartBlocks, kPartFloats / blk_floats) / tiles);
    const int64_t chunks = std::max<int64_t>(1, std::min<int64_t>(steps, cap));
    p.vchunk = (steps + chunks - 1) / chunks * 32;
    p.nz = ceil_div(M, p.vchunk);
    p.bias_off = (int64_t)p.nz * tiles * blk_floats;
    p.part_floats = p.bias_off + (int64_t)p.nz * p.ct * p.rs * 16;
    p.rows = p.nz;
    p.wwidth = tiles * blk_floats;
    p.bwidth = (int64_t)p.ct * p.rs * 16;
    finish_plan(&p);
    return p;
}

// First reduction pass over the partials of plan p, when they have more
// than 2 kRowSlice rows (more than the second pass's lane groups read
// quickly).
// Returns the arguments of the second pass: the partials, or their slice
// sums with rows replaced by slices.
hipError_t sum_slices(const WgradPlan& p, const WgradArgs& a, WgradArgs* b, int64_t* rows,
                      hipStream_t s) {
    *b = a;
    *rows = p.rows;
    if (!p.slices) return hipSuccess;
    const int64_t sl = (p.rows + kRowSlice - 1) / kRowSlice;
    float* out = a.part + p.part_floats;
    hipLaunchKernelGGL(k_sum_row_slices, dim3(ceil_div(sl * (p.wwidth + p.bwidth), 256)),
                       dim3(256), 0, s, (const float*)a.part, p.bias_off, p.rows, p.wwidth,
                       p.bwidth, out);
    b->part = out;
    b->bias_off = sl * p.wwidth;
    *rows = sl;
    return hipGetLastError();
}

}  // namespace

int64_t wgrad_scratch_floats(const ConvGeom& g) {
    return std::max(wgrad_plan(g, 0).scratch_floats, wgrad_plan(g, 1).scratch_floats);
}

// One pass over a brick or 8-cell partial table (rows x W weight entries,
// then the bias rows).
hipError_t launch_partials_sum(const WgradArgs& a, int chunks, int rows, int rs, float* dw,
                               float* db, hipStream_t s) {
    const int64_t W = (int64_t)27 * rs * 16 * 16 * chunks;
    auto blocks = [&](int ent) { return ceil_div(W, ent) + ceil_div(a.cout, ent); };
    if (W >= ((int64_t)1 << 31) || blocks(32) * 32 >= ((int64_t)1 << 31))
        return hipErrorInvalidValue;  // 32-bit entry index
    if (rows <= kPsShortRows)
        hipLaunchKernelGGL((k_brick_partials_sum<1, 256>), dim3((unsigned)blocks(256)), dim3(256), 0,
                           s, a, chunks, rows, rs, dw, db);
    else if (rows >= kPsTallRows && blocks(32) < kPsFewBlocks)
        hipLaunchKernelGGL((k_brick_partials_sum<32, 32>), dim3((unsigned)blocks(32)), dim3(1024), 0,
                           s, a, chunks, rows, rs, dw, db);
    else
        hipLaunchKernelGGL((k_brick_partials_sum<8, 32>), dim3((unsigned)blocks(32)), dim3(256), 0,
                           s, a, chunks, rows, rs, dw, db);
    return hipGetLastError();
}

hipError_t conv_backward_weight(const ConvGeom& g, const __bf16* x1, const __bf16* x2,
                                const __bf16* dy, const __bf16* y, int relu, float* dw,
                                float* db, float* scratch, hipStream_t s) {
    if (!x1 || !dy || !dw || !db || !scratch || (relu && !y) || (g.c2 > 0 && (!x2 || g.lg < 1)))
        return hipErrorInvalidValue;
    const WgradPlan p = wgrad_plan(g, relu);
    WgradArgs a;
    a.x1 = x1;
    a.x2 = x2;
    a.dy = dy;
    a.y = y;
    a.part = scratch;
    a.bias_off = p.bias_off;
    a.n = g.n;
    a.lg = g.lg;
    a.taps = g.taps;
    a.c1 = g.c1;
    a.c1s = g.c1s;
    a.c2 = g.c2;
    a.cin = g.cin;
    a.K = g.K;
    a.cout = g.cout;
    a.coutp = g.coutp;
    a.ys = g.ys;
    a.relu = relu;
    a.cin_real = g.c1 + g.c2;
    a.vchunk = p.vchunk;
    if (p.small) {
        hipLaunchKernelGGL(k_wgrad_small, dim3(p.chunks, g.n, g.coutp / 32), dim3(64 * kWtWaves), 0,
                           s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_partials_sum(a, p.chunks, p.groups, p.rs, dw, db, s);
    }
    if (p.brick) {
        const dim3 grid(p.chunks, p.groups);
        switch (p.rs) {
            case 4: hipLaunchKernelGGL(k_wgrad_brick<4>, grid, dim3(256), 0, s, a, p.per); break;
            case 2: hipLaunchKernelGGL(k_wgrad_tr<2>, grid, dim3(64 * kWtWaves), 0, s, a, p.per); break;
            default: hipLaunchKernelGGL(k_wgrad_tr<1>, grid, dim3(64 * kWtWaves), 0, s, a, p.per); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_partials_sum(a, p.chunks, p.groups, p.rs, dw, db, s);
    }
    const dim3 grid(p.kt, p.ct, p.nz);
    switch (p.rs) {
        case 4: hipLaunchKernelGGL(k_wgrad<4>, grid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_wgrad<2>, grid, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_wgrad<1>, grid, dim3(256), 0, s, a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    WgradArgs b;
    int64_t rows = 0;
    e = sum_slices(p, a, &b, &rows, s);
    if (e != hipSuccess) return e;
    const int64_t nred = (int64_t)p.ct * p.rs * 16 * p.kt * p.cs * 16 + g.cout;
    if (nred * 8 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;  // 32-bit lane index
    if (rows >= kRedManyRows)
        hipLaunchKernelGGL(k_wgrad_reduce<8>, dim3(ceil_div(nred * 8, 256)), dim3(256), 0, s, b,
                           p.kt, p.ct, (int)rows, p.rs, p.cs, dw, db);
    else
        hipLaunchKernelGGL(k_wgrad_reduce<1>, dim3(ceil_div(nred, 256)), dim3(256), 0, s, b, p.kt,
                           p.ct, (int)rows, p.rs, p.cs, dw, db);
    return hipGetLastError();
}

hipError_t pool_forward(int n, int lg, int c, const __bf16* x, __bf16* y, hipStream_t s) {
    if (lg < 1 || c % 8 || !x || !y) return hipErrorInvalidValue;
    const int64_t t = ((int64_t)n << (3 * (lg - 1))) * (c / 8);
    hipLaunchKernelGGL(k_pool, dim3(ceil_div(t, 256)), dim3(256), 0, s, n, lg, c, x, y);
    return hipGetLastError();
}

hipError_t pool_backward_add(int n, int lg, int c, const __bf16* dy, const __bf16* skip, int ctot,
                             const __bf16* ymask, __bf16* dx, hipStream_t s) {
    if (lg < 1 || c % 8 || !dy || !dx || (skip && (ctot < c || ctot % 8))) return hipErrorInvalidValue;
    const int64_t t = ((int64_t)n << (3 * lg)) * (c / 8);
    hipLaunchKernelGGL(k_pool_bwd_add, dim3(ceil_div(t, 256)), dim3(256), 0, s, n, lg, c, dy, skip,
                       ctot, ymask, dx);
    return hipGetLastError();
}

hipError_t upsample_backward(int n, int lg, int c, const __bf16* dcat, int ctot, int coff,
                             const __bf16* ymask, __bf16* dlow, hipStream_t s) {
    if (lg < 1 || c % 8 || coff % 8 || coff + c > ctot || !dcat || !dlow)
        return hipErrorInvalidValue;
    const int64_t t = ((int64_t)n << (3 * (lg - 1))) * (c / 8);
    hipLaunchKernelGGL(k_up_bwd, dim3(ceil_div(t, 256)), dim3(256), 0, s, n, lg, c, dcat, ctot, coff,
                       ymask, dlow);
    return hipGetLastError();
}

hipError_t make_inputs(int n, int lg, const float* log10_ra, __bf16* x, hipStream_t s) {
    if (n < 1 || n > kMaxBatch || !log10_ra || !x) return hipErrorInvalidValue;
    SampleFloats lra;
    for (int i = 0; i < kMaxBatch; ++i) lra.v[i] = i < n ? log10_ra[i] : 0.f;
    const int64_t t = (int64_t)n << (3 * lg);
    hipLaunchKernelGGL(k_inputs, dim3(ceil_div(t, 256)), dim3(256), 0, s, n, lg, lra, x);
    return hipGetLastError();
}

bool head_geometry(const ConvGeom& g) {
    return g.taps == 1 && g.c1 == kHeadIn && g.c1s == kHeadIn && g.c2 == 0 && g.cout == kHeadOut;
}

hipError_t head_forward(const ConvGeom& g, const __bf16* x, const float* w, const float* b,
                        const float* scale4, float* out, hipStream_t s) {
    if (!head_geometry(g) || !x || !w || !b || !out) return hipErrorInvalidValue;
    const float4 sc = scale4 ? make_float4(scale4[0], scale4[1], scale4[2], scale4[3])
                             : make_float4(1.f, 1.f, 1.f, 1.f);
    const int64_t M = (int64_t)g.n << (3 * g.lg);
    hipLaunchKernelGGL(k_head_forward, dim3(ceil_div(M, 256)), dim3(256), 0, s, g.n, g.lg, x, w, b,
                       sc, out);
    return hipGetLastError();
}

int head_backward_blocks(const ConvGeom& g) {
    const int64_t M = (int64_t)g.n << (3 * g.lg);
    return (int)std::min<int64_t>(kHeadBlocks, ceil_div(M, 2048));
}

int64_t head_scratch_floats(const ConvGeom& g) {
    return (int64_t)head_backward_blocks(g) * kHeadGrad;
}

hipError_t head_backward(const ConvGeom& g, const float* targets, const int32_t* idx,
                         int64_t stride, const float* tscale4, const __bf16* x, const float* w,
                         const float* b, __bf16* dx, float* grad, float* scratch,
                         double* lpartial, double* loss, hipStream_t s) {
    if (!head_geometry(g) || g.n < 1 || g.n > kMaxBatch || !targets || !idx || !x || !w || !b ||
        !dx || !grad || !scratch || !lpartial || !loss)
        return hipErrorInvalidValue;
    SampleInts ix;
    for (int i = 0; i < kMaxBatch; ++i) ix.v[i] = i < g.n ? idx[i] : 0;
    const int64_t M = (int64_t)g.n << (3 * g.lg);
    const int nb = head_backward_blocks(g);
    const int64_t chunk = (int64_t)ceil_div(M, (int64_t)nb * 256) * 256;
    const float4 ts = make_float4(tscale4[0], tscale4[1], tscale4[2], tscale4[3]);
    hipLaunchKernelGGL(k_head_backward, dim3(nb), dim3(256), 0, s, g.n, g.lg, targets, ix, stride,
                       ts, x, w, b, chunk, dx, lpartial, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_head_sums, dim3(kHeadGrad + 1), dim3(256), 0, s, (const float*)scratch,
                       nb, kHeadGrad, grad, (const double*)lpartial, loss);
    return hipGetLastError();
}

hipError_t adam_update(int64_t count, float* theta, float* m, float* v, const float* g, int t,
                       float lr, float beta1, float beta2, float eps, hipStream_t s) {
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(ceil_div(count, 256)), dim3(256), 0, s, count, theta, m, v, g,
                       lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t fill_zero_f32(float* p, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(ceil_div(count, 256)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t bf16_to_f32(const __bf16* x, int64_t cells, int cs, int c, float* y, hipStream_t s) {
    const int64_t t = cells * c;
    hipLaunchKernelGGL(k_bf16_to_f32, dim3(ceil_div(t, 256)), dim3(256), 0, s, x, cells, cs, c, y);
    return hipGetLastError();
}

hipError_t cf_to_cl(const float* x, int n, int64_t v, int c, float* y, hipStream_t s) {
    const int64_t t = (int64_t)n * v * c;
    hipLaunchKernelGGL(k_cf_to_cl, dim3(ceil_div(t, 256)), dim3(256), 0, s, x, n, v, c, y);
    return hipGetLastError();
}

}  // namespace lbmnn

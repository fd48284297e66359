// gfx950 kernels of the warm-start network: 3D convolutions as implicit
// GEMMs on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), pooling, upsampling, the loss and Adam.
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
typedef float floatx4 __attribute__((ext_vector_type(4)));

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

struct ConvArgs {
    const __bf16* x1;
    const __bf16* x2;
    const __bf16* mask;
    const __bf16* w;
    const float* bias;
    void* out;
    const __bf16* omask;  // MODE 0: outputs where omask <= 0 are written as 0
    float scale[4];
    int32_t n, lg, taps, c1s, c2, cin, K, kpad, cout, ys, relu;
};

// One block: MT * 16 voxels x (NSUB * 16) output channels, channel group
// blockIdx.y.  Each weight fragment is loaded once and used for the MT
// voxel tiles.  The KS waves of a block split the k range (wave w takes
// every KS-th step of 32 from step w) and add their partial sums through
// LDS; this keeps enough waves in flight on the coarse grids.
template <int NSUB, int MODE, int MT, int KS>
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
    const int kfirst = q * 8 + 32 * wave;
    int tap = kfirst / a.cin, c = kfirst - tap * a.cin;
    for (int k0 = kfirst; k0 < a.kpad; k0 += 32 * KS) {
        int dz = 0, dy = 0, dx = 0;
        if (a.taps == 27) {
            dz = tap / 9 - 1;
            dy = (tap / 3) % 3 - 1;
            dx = tap % 3 - 1;
        }
        bf16x8 av[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int i = 0; i < 8; ++i) av[m][i] = (__bf16)0.f;
            const int zz = vz[m] + dz, yy = vy[m] + dy, xx = vx[m] + dx;
            if (vok[m] && k0 < a.K && (unsigned)zz < (unsigned)G && (unsigned)yy < (unsigned)G &&
                (unsigned)xx < (unsigned)G) {
                if (c < a.c1s) {
                    const int64_t vi = ((int64_t)vs[m] << (3 * lg)) + ((int64_t)zz << (2 * lg)) +
                                       ((int64_t)yy << lg) + xx;
                    av[m] = *(const bf16x8*)(a.x1 + vi * a.c1s + c);
                    if (a.mask) {
                        const bf16x8 mk = *(const bf16x8*)(a.mask + vi * a.c1s + c);
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (!((float)mk[i] > 0.f)) av[m][i] = (__bf16)0.f;
                    }
                } else {
                    const int h = lg - 1;
                    const int64_t vi = ((int64_t)vs[m] << (3 * h)) +
                                       ((int64_t)(zz >> 1) << (2 * h)) +
                                       ((int64_t)(yy >> 1) << h) + (xx >> 1);
                    av[m] = *(const bf16x8*)(a.x2 + vi * a.c2 + (c - a.c1s));
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NSUB; ++j) {
            const bf16x8 bv = *(const bf16x8*)(a.w + (int64_t)(cobase + j * 16 + r) * a.kpad + k0);
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv, acc[m][j], 0, 0, 0);
        }
        c += 32 * KS;
        while (c >= a.cin) c -= a.cin, ++tap;
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
                if (MODE == 0) {
                    if (co < a.ys) {
                        float val = 0.f;
                        if (co < a.cout) {
                            val = acc[m][j][i] + (a.bias ? a.bias[co] : 0.f);
                            if (a.relu) val = fmaxf(val, 0.f);
                            if (a.omask && !((float)a.omask[vo * a.ys + co] > 0.f)) val = 0.f;
                        }
                        ((__bf16*)a.out)[vo * a.ys + co] = (__bf16)val;
                    }
                } else if (co < a.cout) {
                    const float val = acc[m][j][i] + (a.bias ? a.bias[co] : 0.f);
                    const int64_t sidx = vo >> (3 * lg), vin = vo & (V - 1);
                    ((float*)a.out)[(sidx * a.cout + co) * V + vin] = val * a.scale[co];
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
    __shared__ __attribute__((aligned(16))) __bf16 dT[RS * 16][40];
    __shared__ __attribute__((aligned(16))) __bf16 xT[CS * 16][40];
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

// First pass of the partial-sum reduction: out[j][w] = sum of in[g][w] over
// the rows g of slice j (kRowSlice consecutive rows, fewer in the last), in
// order; one thread per (slice, column), so the loads of many rows are in
// flight at once.
constexpr int kRowSlice = 16;
__global__ void k_sum_row_slices(const float* __restrict__ in, int64_t rows, int64_t width,
                                 float* __restrict__ out) {
    const int64_t slices = (rows + kRowSlice - 1) / kRowSlice;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= slices * width) return;
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

// Sum of the k_wgrad partials over the voxel chunks, into the master layout
// dw[co][tap][ci] (zero padding channels dropped) and db.  One thread per
// (row, column) of the gradient matrix or per bias entry.
__global__ void k_wgrad_reduce(WgradArgs a, int kt, int ct, int nz, int rs, int cs, float* dw,
                               float* db) {
    const int64_t rows = (int64_t)ct * rs * 16, cols = (int64_t)kt * cs * 16;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows * cols) {
        const int row = (int)(i / cols), col = (int)(i - (int64_t)row * cols);
        const int cty = row / (rs * 16), rl = row - cty * rs * 16;
        const int ktx = col / (cs * 16), cl = col - ktx * cs * 16;
        if (row >= a.cout || col >= a.K) return;
        const int t = col / a.cin, cc = col - t * a.cin;
        if (cc < a.c1s && cc >= a.c1) return;  // zero padding channels of x1
        const int ci = cc < a.c1s ? cc : a.c1 + (cc - a.c1s);
        const int64_t per = (int64_t)rs * 16 * cs * 16;
        float sum = 0.f;
#pragma unroll 8
        for (int z = 0; z < nz; ++z)
            sum += a.part[(((int64_t)z * ct + cty) * kt + ktx) * per + rl * (cs * 16) + cl];
        dw[((int64_t)row * a.taps + t) * a.cin_real + ci] = sum;
    } else if (i < rows * cols + a.cout) {
        const int co = (int)(i - rows * cols);
        const int cty = co / (rs * 16), rl = co - cty * rs * 16;
        float sum = 0.f;
        for (int z = 0; z < nz; ++z)
            sum += a.part[a.bias_off + ((int64_t)z * ct + cty) * (rs * 16) + rl];
        db[co] = sum;
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
// bias_off).  k_wgrad_brick_reduce adds the partials up.
constexpr int kBrickRow = 4 * 6 * 16 + 8;  // one channel's halo (hz, hy, x), padded

template <int RS>
__global__ void __launch_bounds__(256) k_wgrad_brick(WgradArgs a, int64_t bricks_per_block) {
    constexpr int NT = 7;  // taps per wave: ceil(27 / 4)
    __shared__ __attribute__((aligned(16))) __bf16 xs[3 * 16 * kBrickRow];
    __shared__ __attribute__((aligned(16))) __bf16 dT[RS * 16][136];
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
    bf16x8 reg[10];
    auto fetch = [&](int64_t b) __attribute__((always_inline)) {
        const int x0 = (int)(b % nbx) * 16;
        int64_t rest = b / nbx;
        const int y0 = (int)(rest % nby) * 4;
        rest /= nby;
        const int z0 = (int)(rest % nbz) * 2;
        const int smp = (int)(rest / nbz);
#pragma unroll
        for (int m = 0; m < 10; ++m)
#pragma unroll
            for (int e = 0; e < 8; ++e) reg[m][e] = (__bf16)0.f;
        if (tid < 96) {
            // input halo row (hz, hy), x cells 8k .. 8k+9, channel group cg
            // (the channel group is the slowest index, so the 8 lanes one LDS
            // store cycle serves hit 8 different 4-bank groups)
            const int yy = y0 + hyx - 1, zz = z0 + hzx - 1, cc = c0 + cgx * 8;
            const bool row_ok = cc < a.cin && (unsigned)yy < (unsigned)G && (unsigned)zz < (unsigned)G;
#pragma unroll
            for (int m = 0; m < 10; ++m) {
                const int xx = x0 + 8 * kx + m - 1;
                if (row_ok && (unsigned)xx < (unsigned)G) {
                    if (cc < a.c1s) {
                        const int64_t vi = ((((int64_t)smp << lg) + zz) << (2 * lg)) +
                                           ((int64_t)yy << lg) + xx;
                        reg[m] = *(const bf16x8*)(a.x1 + vi * a.c1s + cc);
                    } else {
                        const int h = lg - 1;
                        const int64_t vi = ((((int64_t)smp << h) + (zz >> 1)) << (2 * h)) +
                                           ((int64_t)(yy >> 1) << h) + (xx >> 1);
                        reg[m] = *(const bf16x8*)(a.x2 + vi * a.c2 + (cc - a.c1s));
                    }
                }
            }
        } else if (tid < 96 + 32 * RS) {
            // output gradient: 8 cells (one k group) x 8 channels
            const int yy = y0 + (sd & 1) * 2 + ((vgd & 3) >> 1), zz = z0 + (sd >> 1);
            const int xb = x0 + (vgd & 1) * 8;
            const int64_t v0 = ((((int64_t)smp << lg) + zz) << (2 * lg)) + ((int64_t)yy << lg) + xb;
            if (cgd * 8 < a.ys) {
#pragma unroll
                for (int m = 0; m < 8; ++m) reg[m] = *(const bf16x8*)(a.dy + (v0 + m) * a.ys + cgd * 8);
            }
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

// Sum of the k_wgrad_brick partials over the brick ranges, into dw[co][tap]
// [ci] (zero padding channels dropped) and db.  One thread per gradient
// entry of (channel group, tap, co, channel) or per bias entry.
__global__ void k_wgrad_brick_reduce(WgradArgs a, int chunks, int groups, int rs, float* dw,
                                     float* db) {
    const int64_t per = (int64_t)27 * rs * 16 * 16;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < per * chunks) {
        const int chunk = (int)(i / per);
        const int e = (int)(i - (int64_t)chunk * per);
        const int t = e / (rs * 256), rem = e - t * rs * 256;
        const int co = rem >> 4, cl = rem & 15;
        const int cc = chunk * 16 + cl;
        if (co >= a.cout || cc >= a.cin || (cc < a.c1s && cc >= a.c1)) return;
        const int ci = cc < a.c1s ? cc : a.c1 + (cc - a.c1s);
        float sum = 0.f;
#pragma unroll 8
        for (int g = 0; g < groups; ++g) sum += a.part[((int64_t)g * chunks + chunk) * per + e];
        dw[((int64_t)co * 27 + t) * a.cin_real + ci] = sum;
    } else if (i < per * chunks + a.cout) {
        const int co = (int)(i - per * chunks);
        float sum = 0.f;
        for (int g = 0; g < groups; ++g) sum += a.part[a.bias_off + (int64_t)g * rs * 16 + co];
        db[co] = sum;
    }
}

__global__ void k_pack_w(int coutp, int kpad, int cout, int K, int cin, int c1, int c1s, int taps,
                         int cin_real, const float* __restrict__ w, __bf16* __restrict__ wp) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)coutp * kpad) return;
    const int co = (int)(idx / kpad), k = (int)(idx - (int64_t)co * kpad);
    float val = 0.f;
    if (co < cout && k < K) {
        const int t = k / cin, cc = k - t * cin;
        if (cc < c1s) {
            if (cc < c1) val = w[((int64_t)co * taps + t) * cin_real + cc];
        } else {
            val = w[((int64_t)co * taps + t) * cin_real + c1 + (cc - c1s)];
        }
    }
    wp[idx] = (__bf16)val;
}

__global__ void k_pack_wt(int cinp, int kpad_t, int cin, int ys, int cout, int c1, int c1s,
                          int taps, int cin_real, const float* __restrict__ w,
                          __bf16* __restrict__ wt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)cinp * kpad_t) return;
    const int ci = (int)(idx / kpad_t), k = (int)(idx - (int64_t)ci * kpad_t);
    float val = 0.f;
    if (ci < cin && k < taps * ys) {
        const int t = k / ys, co = k - t * ys;
        const bool real = ci >= c1s || ci < c1;
        if (co < cout && real) {
            const int cir = ci < c1s ? ci : c1 + (ci - c1s);
            val = w[((int64_t)co * taps + (taps - 1 - t)) * cin_real + cir];
        }
    }
    wt[idx] = (__bf16)val;
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

__global__ void __launch_bounds__(256) k_mse(int n, int lg, const float* __restrict__ out,
                                             const float* __restrict__ tg, SampleInts idx,
                                             int64_t stride,
                                             float4 ts, __bf16* __restrict__ dy,
                                             double* __restrict__ partial) {
    __shared__ double red[256];
    const int64_t V = (int64_t)1 << (3 * lg);
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double inv = 2.0 / ((double)n * 4.0 * (double)V);
    double acc = 0.0;
    if (v < (int64_t)n * V) {
        const int s = (int)(v >> (3 * lg));
        const int64_t vin = v & (V - 1);
        const float tsc[4] = {ts.x, ts.y, ts.z, ts.w};
        bf16x8 o;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float ov = out[((int64_t)s * 4 + c) * V + vin];
            const float tv = tg[(int64_t)idx.v[s] * stride + c * V + vin] * tsc[c];
            const double d = (double)ov - (double)tv;
            acc += d * d;
            o[c] = (__bf16)(float)(d * inv);
        }
        o[4] = o[5] = o[6] = o[7] = (__bf16)0.f;
        *(bf16x8*)(dy + v * 8) = o;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) k_reduce(const double* __restrict__ p, int n,
                                                 double* __restrict__ out) {
    __shared__ double red[1024];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc += p[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
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
// BF16 output, grids of at least 16 cells, input channels a multiple of
// 16).  A block of 8 waves computes 16 x 4 x 8 output voxels (wave w the
// plane z0 + w, its four 16-voxel row tiles y0 .. y0 + 3) for NSUB * 16
// output channels.  Per 16 input channels the block stages the 18 x 6 x 10
// input halo channels-last in LDS (48 bytes per voxel: 16 channels and 8 of
// padding, which puts the 16-byte reads of 8 consecutive lanes on distinct
// banks), so every A fragment (8 channels of one voxel for one tap) is one
// LDS read instead of a global load per tap.  A k step of 32 pairs two taps
// of the 16 channels; B fragments are read from the packed weight ([co][k],
// k = tap * cin + channel) and serve the four row tiles.
constexpr int kCvVox = 24;                  // LDS elements per voxel
constexpr int kCvPlanes = 8;                // output planes (waves) per block
constexpr int kCvHalo = 18 * 6 * (kCvPlanes + 2);  // halo voxels

template <int NSUB>
__global__ void __launch_bounds__(64 * kCvPlanes) k_conv_brick(ConvArgs a) {
    __shared__ __attribute__((aligned(16))) __bf16 xs[kCvHalo * kCvVox];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int lg = a.lg, G = 1 << lg;
    const int nbx = G >> 4, nby = G >> 2, nbz = G / kCvPlanes;
    int64_t bid = blockIdx.x;
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
    for (int c0 = 0; c0 < a.cin; c0 += 16) {
        for (int t = tid; t < 2 * kCvHalo; t += 64 * kCvPlanes) {
            const int half = t & 1, hv = t >> 1;
            const int hx = hv % 18, hy = (hv / 18) % 6, hz = hv / 108;
            const int xx = x0 + hx - 1, yy = y0 + hy - 1, zz = z0 + hz - 1;
            const int cc = c0 + half * 8;
            bf16x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.f;
            if ((unsigned)xx < (unsigned)G && (unsigned)yy < (unsigned)G &&
                (unsigned)zz < (unsigned)G) {
                if (cc < a.c1s) {
                    const int64_t vi = ((((int64_t)smp << lg) + zz) << (2 * lg)) +
                                       ((int64_t)yy << lg) + xx;
                    v = *(const bf16x8*)(a.x1 + vi * a.c1s + cc);
                } else {
                    const int h = lg - 1;
                    const int64_t vi = ((((int64_t)smp << h) + (zz >> 1)) << (2 * h)) +
                                       ((int64_t)(yy >> 1) << h) + (xx >> 1);
                    v = *(const bf16x8*)(a.x2 + vi * a.c2 + (cc - a.c1s));
                }
            }
            *(bf16x8*)&xs[hv * kCvVox + half * 8] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int p = 0; p < 14; ++p) {
            const int t = 2 * p + (q >> 1);  // this lane's tap
            bf16x8 bv[NSUB];
            bf16x8 av[4];
            if (t < 27) {
                const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
#pragma unroll
                for (int j = 0; j < NSUB; ++j)
                    bv[j] = *(const bf16x8*)(a.w + (int64_t)(cobase + j * 16 + r) * a.kpad +
                                             t * a.cin + c0 + ch);
                const int base = ((wave + dz + 1) * 6 + dy + 1) * 18 + r + dx + 1;
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    av[m] = *(const bf16x8*)&xs[(base + m * 18) * kCvVox + ch];
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
#pragma unroll
                    for (int j = 0; j < NSUB; ++j) bv[j][e] = (__bf16)0.f;
#pragma unroll
                    for (int m = 0; m < 4; ++m) av[m][e] = (__bf16)0.f;
                }
            }
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
                    ((__bf16*)a.out)[vo * a.ys + co] = (__bf16)val;
                }
            }
        }
    }
}

template <int MODE, int MT, int KS>
hipError_t launch_conv_mt(const ConvArgs& a, int coutp, hipStream_t s) {
    const int64_t M = (int64_t)a.n << (3 * a.lg);
    const int sub = coutp / 16;
    const int nsub = sub % 4 == 0 ? 4 : sub % 3 == 0 ? 3 : sub % 2 == 0 ? 2 : 1;
    const dim3 grid(ceil_div(M, 16 * MT), sub / nsub), block(64 * KS);
    switch (nsub) {
        case 4: hipLaunchKernelGGL((k_conv<4, MODE, MT, KS>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_conv<3, MODE, MT, KS>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_conv<2, MODE, MT, KS>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((k_conv<1, MODE, MT, KS>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

// Four voxel tiles per wave when that still leaves at least 2048 blocks (so
// each weight fragment serves 64 voxels).  Otherwise one tile, and the k
// range is split over 2 or 4 waves per block when there are fewer than
// 4096 or 1024 blocks and at least two steps of 32 per wave.
template <int MODE>
hipError_t launch_conv(const ConvArgs& a, int coutp, hipStream_t s) {
    const int64_t M = (int64_t)a.n << (3 * a.lg);
    const int sub = coutp / 16;
    const int nsub = sub % 4 == 0 ? 4 : sub % 3 == 0 ? 3 : sub % 2 == 0 ? 2 : 1;
    if (MODE == 0 && a.taps == 27 && a.lg >= 4 && a.cin % 16 == 0 && !a.mask &&
        a.kpad >= 27 * a.cin) {
        // on the 16-cell grid one output-channel group per block, for blocks
        const int64_t G = (int64_t)1 << a.lg;
        const int nb = a.lg >= 5 ? nsub : 1;
        const dim3 grid((unsigned)((G / 16) * (G / 4) * (G / kCvPlanes) * a.n), sub / nb);
        const dim3 block(64 * kCvPlanes);
        switch (nb) {
            case 4: hipLaunchKernelGGL(k_conv_brick<4>, grid, block, 0, s, a); break;
            case 3: hipLaunchKernelGGL(k_conv_brick<3>, grid, block, 0, s, a); break;
            case 2: hipLaunchKernelGGL(k_conv_brick<2>, grid, block, 0, s, a); break;
            default: hipLaunchKernelGGL(k_conv_brick<1>, grid, block, 0, s, a); break;
        }
        return hipGetLastError();
    }
    const int64_t waves4 = (int64_t)ceil_div(M, 64) * (sub / nsub);
    if (waves4 >= 2048) return launch_conv_mt<MODE, 4, 1>(a, coutp, s);
    const int64_t waves1 = (int64_t)ceil_div(M, 16) * (sub / nsub);
    const int ksteps = a.kpad / 32;
    if (waves1 < 1024 && ksteps >= 8) return launch_conv_mt<MODE, 1, 4>(a, coutp, s);
    if (waves1 < 4096 && ksteps >= 4) return launch_conv_mt<MODE, 1, 2>(a, coutp, s);
    return launch_conv_mt<MODE, 1, 1>(a, coutp, s);
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

hipError_t pack_weights(const ConvGeom& g, const float* w, __bf16* wp, __bf16* wt,
                        hipStream_t s) {
    const int cin_real = g.c1 + g.c2;
    const int64_t n1 = (int64_t)g.coutp * g.kpad;
    hipLaunchKernelGGL(k_pack_w, dim3(ceil_div(n1, 256)), dim3(256), 0, s, g.coutp, g.kpad, g.cout,
                       g.K, g.cin, g.c1, g.c1s, g.taps, cin_real, w, wp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !wt) return e;
    const int64_t n2 = (int64_t)g.cinp * g.kpad_t;
    hipLaunchKernelGGL(k_pack_wt, dim3(ceil_div(n2, 256)), dim3(256), 0, s, g.cinp, g.kpad_t, g.cin,
                       g.ys, g.cout, g.c1, g.c1s, g.taps, cin_real, w, wt);
    return hipGetLastError();
}

hipError_t conv_forward(const ConvGeom& g, const __bf16* x1, const __bf16* x2,
                        const __bf16* mask, const __bf16* wp, const float* bias, int relu,
                        int mode, void* out, const float* scale4, hipStream_t s) {
    if (!x1 || !wp || !out || (g.c2 > 0 && (!x2 || g.lg < 1)) || g.c1s % 8 || g.c2 % 8 ||
        (mode == 1 && g.cout > 4))
        return hipErrorInvalidValue;
    ConvArgs a;
    a.x1 = x1;
    a.x2 = x2;
    a.mask = mask;
    a.w = wp;
    a.bias = bias;
    a.out = out;
    a.omask = nullptr;
    for (int i = 0; i < 4; ++i) a.scale[i] = scale4 ? scale4[i] : 1.f;
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
    return mode == 0 ? launch_conv<0>(a, g.coutp, s) : launch_conv<1>(a, g.coutp, s);
}

hipError_t conv_backward_data(const ConvGeom& g, const __bf16* dy, const __bf16* wt,
                              const __bf16* dxmask, __bf16* dx, hipStream_t s) {
    if (!dy || !wt || !dx) return hipErrorInvalidValue;
    ConvArgs a;
    a.x1 = dy;
    a.x2 = nullptr;
    a.mask = nullptr;
    a.w = wt;
    a.bias = nullptr;
    a.out = dx;
    a.omask = dxmask;
    for (int i = 0; i < 4; ++i) a.scale[i] = 1.f;
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
    return launch_conv<0>(a, g.cinp, s);
}

namespace {

// Launch plan of the weight gradient: the brick kernel (grids of at least 16
// cells, 27 taps, >= 16 input channels, 16/32/64 output channels) or the
// tiled kernel, its grid, and the floats of partial sums it writes.
struct WgradPlan {
    bool brick;
    int rs, cs;
    int chunks, groups;  // brick: channel groups x brick ranges
    int64_t per;         // brick: bricks per range
    int kt, ct, nz;      // tiled: column tiles, row tiles, voxel chunks
    int64_t vchunk;
    int64_t part_floats, bias_off;  // partial sums of every block
    int64_t rows, wwidth, bwidth;   // rows of partials, weight / bias floats per row
    int64_t scratch_floats;         // partials + the first reduction pass
};

// Scratch of the first reduction pass, after the partials: the weight rows
// and the bias rows summed over slices of kRowSlice rows.
void finish_plan(WgradPlan* p) {
    const int64_t sl = (p->rows + kRowSlice - 1) / kRowSlice;
    p->scratch_floats = p->part_floats + sl * (p->wwidth + p->bwidth);
}

// Partial sums kept to about 32 MB and 1024 blocks: enough blocks to fill
// the chip, and a second pass that reads far less than the layer's inputs.
constexpr int64_t kPartFloats = 8 << 20;
constexpr int64_t kPartBlocks = 1024;

// (The brick kernel reads the output gradient unmasked: relu != 0 takes the
// tiled kernel.)
WgradPlan wgrad_plan(const ConvGeom& g, int relu) {
    WgradPlan p = {};
    const int64_t M = (int64_t)g.n << (3 * g.lg);
    p.brick = !relu && g.lg >= 4 && g.taps == 27 && g.cin >= 16 &&
              (g.coutp == 16 || g.coutp == 32 || g.coutp == 64);
    if (p.brick) {
        p.rs = g.coutp / 16;
        p.chunks = ceil_div(g.cin, 16);
        const int64_t nbricks = M / 128;
        const int64_t blk_floats = (int64_t)27 * g.coutp * 16;
        const int64_t cap = std::max<int64_t>(
            1, std::min<int64_t>(kPartBlocks, kPartFloats / blk_floats) / p.chunks);
        const int64_t groups = std::max<int64_t>(1, std::min<int64_t>(nbricks, cap));
        p.per = (nbricks + groups - 1) / groups;
        p.groups = ceil_div(nbricks, p.per);
        p.bias_off = (int64_t)p.groups * p.chunks * blk_floats;
        p.part_floats = p.bias_off + (int64_t)p.groups * g.coutp;
        p.rows = p.groups;
        p.wwidth = (int64_t)p.chunks * blk_floats;
        p.bwidth = g.coutp;
        finish_plan(&p);
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

// First reduction pass over the partials of plan p; returns the arguments
// of the second pass (partials replaced by the slice sums, rows by slices).
hipError_t sum_slices(const WgradPlan& p, const WgradArgs& a, WgradArgs* b, int64_t* rows,
                      hipStream_t s) {
    const int64_t sl = (p.rows + kRowSlice - 1) / kRowSlice;
    float* out = a.part + p.part_floats;
    hipLaunchKernelGGL(k_sum_row_slices, dim3(ceil_div(sl * p.wwidth, 256)), dim3(256), 0, s,
                       (const float*)a.part, p.rows, p.wwidth, out);
    hipLaunchKernelGGL(k_sum_row_slices, dim3(ceil_div(sl * p.bwidth, 256)), dim3(256), 0, s,
                       (const float*)(a.part + p.bias_off), p.rows, p.bwidth,
                       out + sl * p.wwidth);
    *b = a;
    b->part = out;
    b->bias_off = sl * p.wwidth;
    *rows = sl;
    return hipGetLastError();
}

}  // namespace

int64_t wgrad_scratch_floats(const ConvGeom& g) {
    return std::max(wgrad_plan(g, 0).scratch_floats, wgrad_plan(g, 1).scratch_floats);
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
    if (p.brick) {
        const dim3 grid(p.chunks, p.groups);
        switch (p.rs) {
            case 4: hipLaunchKernelGGL(k_wgrad_brick<4>, grid, dim3(256), 0, s, a, p.per); break;
            case 2: hipLaunchKernelGGL(k_wgrad_brick<2>, grid, dim3(256), 0, s, a, p.per); break;
            default: hipLaunchKernelGGL(k_wgrad_brick<1>, grid, dim3(256), 0, s, a, p.per); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        WgradArgs b;
        int64_t rows = 0;
        e = sum_slices(p, a, &b, &rows, s);
        if (e != hipSuccess) return e;
        const int64_t nred = (int64_t)27 * g.coutp * 16 * p.chunks + g.cout;
        hipLaunchKernelGGL(k_wgrad_brick_reduce, dim3(ceil_div(nred, 256)), dim3(256), 0, s, b,
                           p.chunks, (int)rows, p.rs, dw, db);
        return hipGetLastError();
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
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(ceil_div(nred, 256)), dim3(256), 0, s, b, p.kt, p.ct,
                       (int)rows, p.rs, p.cs, dw, db);
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

hipError_t mse_forward_backward(int n, int lg, const float* out, const float* targets,
                                const int32_t* idx, int64_t stride, const float* tscale4,
                                __bf16* dy, double* partial, int* nblocks, hipStream_t s) {
    if (n < 1 || n > kMaxBatch || !out || !targets || !idx || !dy || !partial)
        return hipErrorInvalidValue;
    SampleInts ix;
    for (int i = 0; i < kMaxBatch; ++i) ix.v[i] = i < n ? idx[i] : 0;
    const int64_t t = (int64_t)n << (3 * lg);
    const int nb = ceil_div(t, 256);
    *nblocks = nb;
    const float4 ts = make_float4(tscale4[0], tscale4[1], tscale4[2], tscale4[3]);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, n, lg, out, targets, ix, stride, ts, dy,
                       partial);
    return hipGetLastError();
}

hipError_t reduce_sum(const double* partial, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, partial, n, out);
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

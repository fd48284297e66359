// Host-side declarations shared by the warm-start network driver
// (nn_net.cpp) and its kernels (nn_kernels.hip).  Not part of the public
// interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmnn {

constexpr int kMaxBatch = 64;  // samples per call

// One convolution over n samples on a cubic grid of edge 2^lg.  The input
// is the channel concatenation of x1 (c1s stored channels on this grid, of
// which c1 are real; the rest hold zeros) and, when c2 > 0, x2 (c2 channels
// on the grid of edge 2^(lg-1), read through nearest-neighbour upsampling).
struct ConvGeom {
    int32_t n, lg;
    int32_t taps;       // 27 (3x3x3) or 1 (1x1x1)
    int32_t c1, c1s, c2;
    int32_t cin;        // c1s + c2: stored input channels, K per tap
    int32_t K, kpad;    // taps * cin, rounded up to 32
    int32_t cout;       // real output channels
    int32_t coutp;      // rows of the packed weight: cout rounded up to 16
    int32_t ys;         // stored channels of the output and its gradient: cout rounded up to 8
    int32_t kpad_t;     // columns of the transposed weight: taps * ys rounded up to 32
    int32_t cinp;       // rows of the transposed weight: cin rounded up to 16
};

ConvGeom make_geom(int n, int lg, int taps, int c1, int c2, int cout);

// Master weights of layer l at theta + woff[l], w[co][tap][ci] (ci over the
// c1 + c2 real channels) -> packed BF16 rows wp[l][coutp][kpad] (k = tap *
// cin + stored channel) and the transposed, tap-flipped copy
// wt[l][cinp][kpad_t] (k = tap * ys + co) that turns the input gradient into
// a forward convolution; all layers (at most kMaxPackLayers) in one launch.
constexpr int kMaxPackLayers = 16;
hipError_t pack_weights(int layers, const ConvGeom* g, const float* theta, const int64_t* woff,
                        __bf16* const* wp, __bf16* const* wt, hipStream_t s);

// Device FP32 scratch a convolution of geometry g may use (forward or input
// gradient): 8-cell grids split the products over the input channel groups
// and keep partial sums there.  0 when no launch needs any.
int64_t conv_scratch_floats(const ConvGeom& g);

// out = conv(x1, x2) + bias, ReLU if relu; BF16 channels-last [n][v][ys].
// scratch: scratch_floats device floats (conv_scratch_floats(g) or more), or
// null (the tiled kernel then runs on 8-cell grids).
hipError_t conv_forward(const ConvGeom& g, const __bf16* x1, const __bf16* x2, const __bf16* wp,
                        const float* bias, int relu, __bf16* out, float* scratch,
                        int64_t scratch_floats, hipStream_t s);

// Input gradient: dx[n][v][cin] = sum over taps and co of dy at the
// neighbour times the weight.  dy is the gradient of the pre-activation
// (already masked by the ReLU).  When dxmask is given (the ReLU output of
// the layer that produced x), dx is written as 0 where dxmask <= 0, so the
// result is again a pre-activation gradient.
hipError_t conv_backward_data(const ConvGeom& g, const __bf16* dy, const __bf16* wt,
                              const __bf16* dxmask, __bf16* dx, float* scratch,
                              int64_t scratch_floats, hipStream_t s);

// Weight and bias gradients, written into the master layout:
// dw[co][tap][ci] = sum_v dpre[v][co] x(v + tap)[ci], db[co] = sum_v
// dpre[v][co] (dpre = dy, masked by y > 0 when relu).  Blocks sum ranges of
// voxels into scratch (wgrad_scratch_floats(g) floats, device), a second
// kernel adds the ranges in a fixed order.
int64_t wgrad_scratch_floats(const ConvGeom& g);
hipError_t conv_backward_weight(const ConvGeom& g, const __bf16* x1, const __bf16* x2,
                                const __bf16* dy, const __bf16* y, int relu, float* dw,
                                float* db, float* scratch, hipStream_t s);

// Average pooling of 2x2x2 blocks: x on grid 2^lg, y on 2^(lg-1), c channels.
hipError_t pool_forward(int n, int lg, int c, const __bf16* x, __bf16* y, hipStream_t s);
// dx (grid 2^lg) = dy_coarse(parent) / 8 + skip[v][0..c) (skip has ctot
// channels per cell; NULL adds nothing), set to 0 where ymask <= 0 (ymask:
// [v][c], may be NULL).
hipError_t pool_backward_add(int n, int lg, int c, const __bf16* dy, const __bf16* skip, int ctot,
                             const __bf16* ymask, __bf16* dx, hipStream_t s);
// dlow (grid 2^(lg-1)) = sum over the 8 children of dcat[child][coff..coff+c),
// set to 0 where ymask <= 0 (ymask: [v][c] on the coarse grid, may be NULL).
hipError_t upsample_backward(int n, int lg, int c, const __bf16* dcat, int ctot, int coff,
                             const __bf16* ymask, __bf16* dlow, hipStream_t s);

// Network input [n][v][8] (BF16): (log10 Ra - 4)/2, x, y, z, 0, 0, 0, 0;
// log10_ra is a host array of n <= kMaxBatch values (passed by value).
hipError_t make_inputs(int n, int lg, const float* log10_ra, __bf16* x, hipStream_t s);

// The 1 x 1 x 1 head (16 BF16 input channels -> 4 FP32 outputs) on the
// vector units with the FP32 master weights w[co][ci] and bias b[co]:
// out[n][4][v] (channel-first) = (w x + b) * scale4[c] (scale4 NULL: 1).
bool head_geometry(const ConvGeom& g);
hipError_t head_forward(const ConvGeom& g, const __bf16* x, const float* w, const float* b,
                        const float* scale4, float* out, hipStream_t s);
// Loss and backward step of the head in one pass over the voxels, its output
// out = w x + b computed on the way (as head_forward computes it): against
// targets[idx[i]] (channel-first, stride floats apart, times tscale4), the
// output gradient 2 (out - t) / count, the input gradient dx[n][v][16]
// (BF16, 0 where x <= 0), the weight and bias gradients (grad: w[4][16] then
// b[4], FP32) and the summed squared error (*loss, device, FP64).  Scratch:
// head_scratch_floats(g) floats and head_backward_blocks(g) doubles at
// lpartial.  Sums run in a fixed order.
constexpr int kHeadBlocks = 1024;
int head_backward_blocks(const ConvGeom& g);
int64_t head_scratch_floats(const ConvGeom& g);
hipError_t head_backward(const ConvGeom& g, const float* targets, const int32_t* idx,
                         int64_t stride, const float* tscale4, const __bf16* x, const float* w,
                         const float* b, __bf16* dx, float* grad, float* scratch,
                         double* lpartial, double* loss, hipStream_t s);

hipError_t adam_update(int64_t count, float* theta, float* m, float* v, const float* g, int t,
                       float lr, float beta1, float beta2, float eps, hipStream_t s);
hipError_t fill_zero_f32(float* p, int64_t count, hipStream_t s);
// BF16 channels-last [n][v][cs] (first c channels) -> FP32 [n][v][c].
hipError_t bf16_to_f32(const __bf16* x, int64_t cells, int cs, int c, float* y, hipStream_t s);
// FP32 channel-first [n][c][v] -> channels-last [n][v][c].
hipError_t cf_to_cl(const float* x, int n, int64_t v, int c, float* y, hipStream_t s);

}  // namespace lbmnn

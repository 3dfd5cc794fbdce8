// Declarations shared by the learned warm start (cnn.hip, cnn_kernels.hip).
#pragma once

#include <cstdint>

#include "ew_internal.h"

namespace ew {

constexpr int kCnnParams = EW_CNN_PARAMS;
// offsets in the parameter vector: W1[16][4][3][3], b1, W2[16][16][3][3], b2, W3[16][3][3], b3
constexpr int kOffW1 = 0, kOffB1 = 576, kOffW2 = 592, kOffB2 = 2896, kOffW3 = 2912, kOffB3 = 3056;
constexpr int kCnnHalo = EW_CNN_HALO;
constexpr int kCnnTrainBlocks = 1024;  // upper bound of the training grid (one gradient partial per block)

// Parameter image used by the kernels, rebuilt from the FP32 master after
// every change.  The MFMA A-operand fragments hold BF16 bits in lane order of
// v_mfma_f32_16x16x16_bf16 (lane l: row l % 16, k = 4 (l / 16) + 0..3).
struct CnnPacked {
    uint16_t w1[3][64][4];   // layer 1: A[o][k], k = 4 tap + channel (taps >= 9 are zero)
    uint16_t w2[9][64][4];   // layer 2, per tap: A[o][c]
    uint16_t w2t[9][64][4];  // layer 2 transposed, per tap: A[c][o] (backward through layer 2)
    float b1[16];
    float b2[16];
    float w3[144];           // layer 3, [c][tap], BF16-rounded values
    float b3;
    float pad[3];
};

// One training crop: constant planes, the half-open rectangle of the padded
// window that lies inside the grid (a window edge on the grid's boundary is a
// wall), and the step's operator M = I - a L_h in units of the spacing:
// a / h_x^2, a / h_y^2 and the stencil order.
struct CropMeta {
    float c2, c3;
    int r0, r1, c0, c1;
    float ahx, ahy;
    int order;
    int pad;
};

hipError_t launch_cnn_pack(const float* params, CnnPacked* pk, hipStream_t s);

// x += s y over an nx x ny grid, y the network output on the planes
// (r / s, b * b_scale, c2, c3); s = sqrt(sum of the kRedBlocks partials of
// r^2 * inv_n) is read on the device (a zero residual leaves x unchanged).
hipError_t launch_cnn_infer(const CnnPacked* pk, const double* r, const double* b, double* x, int nx, int ny,
                            const double* r2_partials, double inv_n, double b_scale, float c2, float c3,
                            hipStream_t st);

// Crops from one implicit step: for crop j with window origin (oy[j], ox[j]),
// fields (r * inv_s, b * b_scale) over the padded window and target
// r * inv_s over the window.
hipError_t launch_cnn_extract(const double* r, const double* b, int nx, int ny, double inv_s, double b_scale,
                              const int* origins_dev, int ncrop, int crop, float* fields_out, float* target_out,
                              hipStream_t st);

// Over the crops ids[0..count): mode 0 writes y_out; mode 1 writes per-block
// partial gradients (pgrad[block][kCnnParams]) from dL/dy = dy_in and loss
// partials sum e_in^2 * inv_npix (dy_in, e_in: [count][crop][crop]).
hipError_t launch_cnn_train(const CnnPacked* pk, const float* fields, const CropMeta* meta, const int* ids,
                            int count, int crop, int mode, float* y_out, const float* dy_in, const float* e_in,
                            float inv_npix, float* pgrad, double* ploss, int nblocks, hipStream_t st);

// Residual loss of the residual form on the crops ids[0..count) with network
// outputs y ([count][crop][crop]): e = target - M y on the loss points (every
// stencil neighbour inside the window or beyond a wall, the wall closures of
// L_h applied), 0 elsewhere; then dy = -2 inv_npix M e (M is symmetric).
hipError_t launch_cnn_resloss(const float* y, const float* target, const CropMeta* meta, const int* ids, int count,
                              int crop, float inv_npix, float* e_out, float* dy_out, hipStream_t st);
int cnn_train_blocks(int count, int crop);

// grad[i] = sum over blocks of pgrad[b][i]; *loss = sum of ploss (fixed order).
hipError_t launch_cnn_reduce(const float* pgrad, const double* ploss, int nblocks, float* grad, double* loss,
                             hipStream_t st);

// One Adam update of the FP32 master (bias corrections inv_c1 = 1/(1-beta1^t),
// inv_c2 = 1/(1-beta2^t)) followed by the repack.
hipError_t launch_cnn_adam_pack(float* params, float* m, float* v, const float* grad, float lr, float beta1,
                                float beta2, float eps, float inv_c1, float inv_c2, CnnPacked* pk, hipStream_t st);

}  // namespace ew

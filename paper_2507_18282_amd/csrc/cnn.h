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

// One training crop: constant planes and the half-open rectangle of the
// padded window that lies inside the grid.
struct CropMeta {
    float c2, c3;
    int r0, r1, c0, c1;
};

hipError_t launch_cnn_pack(const float* params, CnnPacked* pk, hipStream_t s);

// guess = base_scale * wn + s * y over an nx x ny grid, y the network output
// on the planes (wn * inv_s, wprev * inv_s, c2, c3).
hipError_t launch_cnn_infer(const CnnPacked* pk, const double* wn, const double* wprev, double* guess, int nx,
                            int ny, double inv_s, double s, double base_scale, float c2, float c3, hipStream_t st);

// Crops from one implicit step: for crop j with window origin (oy[j], ox[j]),
// fields (W^n, W^{n-1}) * inv_s over the padded window and target
// (S - base_scale W^n) * inv_s over the window.
hipError_t launch_cnn_extract(const double* wn, const double* wprev, const double* S, int nx, int ny,
                              double inv_s, double base_scale, const int* origins_dev, int ncrop, int crop,
                              float* fields_out, float* target_out, hipStream_t st);

// Over the crops ids[0..count): mode 0 writes y_out; mode 1 writes per-block
// partial gradients (pgrad[block][kCnnParams]) and loss partials.
hipError_t launch_cnn_train(const CnnPacked* pk, const float* fields, const float* target, const CropMeta* meta,
                            const int* ids, int count, int crop, int mode, float* y_out, float inv_npix,
                            float* pgrad, double* ploss, int nblocks, hipStream_t st);
int cnn_train_blocks(int count, int crop);

// grad[i] = sum over blocks of pgrad[b][i]; *loss = sum of ploss (fixed order).
hipError_t launch_cnn_reduce(const float* pgrad, const double* ploss, int nblocks, float* grad, double* loss,
                             hipStream_t st);

// One Adam update of the FP32 master (bias corrections inv_c1 = 1/(1-beta1^t),
// inv_c2 = 1/(1-beta2^t)) followed by the repack.
hipError_t launch_cnn_adam_pack(float* params, float* m, float* v, const float* grad, float lr, float beta1,
                                float beta2, float eps, float inv_c1, float inv_c2, CnnPacked* pk, hipStream_t st);

}  // namespace ew

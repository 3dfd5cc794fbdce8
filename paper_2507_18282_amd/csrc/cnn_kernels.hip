// Kernels of the learned warm start.  The 3-layer 3x3 network runs on LDS
// tiles: layers 1 and 2 (and the backward pass through layer 2 and the
// weight gradients) are BF16 v_mfma_f32_16x16x16_bf16 products with FP32
// accumulation, layer 3 and the elementwise parts run on the vector ALUs.
//
// Tile frames (row-major, x fastest) for an output tile of TH x TW points:
//   X  (TH+6) x (TW+6)  input planes, 4 BF16 channels per point (8 B)
//   A1 (TH+4) x (TW+4)  layer-1 activations, 16 BF16 channels (32 B)
//   A2 (TH+2) x (TW+2)  layer-2 activations, 16 BF16 channels (32 B)
// Every convolution is "valid" inside the tile, so a tile recomputes the
// activations of its halo and tiles never exchange data.
//
// MFMA operand layout (16x16x16, 64 lanes): lane l holds A[l % 16][k] and
// B[k][l % 16] for k = 4 (l / 16) + 0..3, and D[4 (l / 16) + 0..3][l % 16].
// For a convolution the A operand is a weight matrix A[o][c] held in
// registers for the whole kernel and B[c][p] is 16 consecutive frame points
// p, each lane reading the 4 channels 4 (l / 16).. of its own point (8 B).
#include "cnn.h"
#include "stencil_dev.h"

namespace ew {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint32_t bf_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf_val(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ u32x2 pack_bf4(float a, float b, float c, float d) {
    u32x2 r;
    r.x = bf_bits(a) | (bf_bits(b) << 16);
    r.y = bf_bits(c) | (bf_bits(d) << 16);
    return r;
}
__device__ __forceinline__ bf16x4 frag(u32x2 v) { return __builtin_bit_cast(bf16x4, v); }
__device__ __forceinline__ bf16x4 frag4(const uint32_t (&h)[4]) {
    u32x2 r;
    r.x = h[0] | (h[1] << 16);
    r.y = h[2] | (h[3] << 16);
    return frag(r);
}
__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 zero4() {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
}

template <int TH, int TW>
struct TileGeo {
    static constexpr int OH = TH, OW = TW, NO = TH * TW;
    static constexpr int XW = TW + 6, XH = TH + 6, NXP = XW * XH;
    static constexpr int AW1 = TW + 4, AH1 = TH + 4, N1 = AW1 * AH1;
    static constexpr int AW2 = TW + 2, AH2 = TH + 2, N2 = AW2 * AH2;
};

// Per-lane weight fragments and biases.
struct LaneWeights {
    bf16x4 w1[3];
    bf16x4 w2[9];
    float bias1[4], bias2[4];
};

__device__ __forceinline__ void load_lane_weights(const CnnPacked* __restrict__ pk, int lane, LaneWeights& w) {
    const int grp = lane >> 4;
#pragma unroll
    for (int t = 0; t < 3; ++t) w.w1[t] = frag(reinterpret_cast<const u32x2*>(pk->w1[t])[lane]);
#pragma unroll
    for (int t = 0; t < 9; ++t) w.w2[t] = frag(reinterpret_cast<const u32x2*>(pk->w2[t])[lane]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        w.bias1[r] = pk->b1[4 * grp + r];
        w.bias2[r] = pk->b2[4 * grp + r];
    }
}

// Layer 1: X (4 channels) -> A1 (16 channels), K = 4 tap + channel, 3 MFMAs
// per 16 points.
template <class G, int NW>
__device__ __forceinline__ void conv1(const u32x2* __restrict__ xs, u32x2* __restrict__ a1, const LaneWeights& w,
                                      int wave, int lane) {
    const int grp = lane >> 4, col = lane & 15;
    int off[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int tap = 4 * t + grp;
        off[t] = tap < 9 ? (tap / 3) * G::XW + tap % 3 : -1;
    }
    for (int g = wave; g * 16 < G::N1; g += NW) {
        const int p = g * 16 + col;
        const int pc = p < G::N1 ? p : G::N1 - 1;
        const int py = pc / G::AW1;
        const int base = py * G::XW + (pc - py * G::AW1);
        f32x4 acc = zero4();
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            u32x2 v = xs[off[t] >= 0 ? base + off[t] : 0];
            if (off[t] < 0) v = u32x2{0u, 0u};
            acc = mfma(w.w1[t], frag(v), acc);
        }
        if (p < G::N1)
            a1[p * 4 + grp] = pack_bf4(fmaxf(acc[0] + w.bias1[0], 0.f), fmaxf(acc[1] + w.bias1[1], 0.f),
                                       fmaxf(acc[2] + w.bias1[2], 0.f), fmaxf(acc[3] + w.bias1[3], 0.f));
    }
}

// Layer 2: A1 -> A2, one MFMA per tap per 16 points.
template <class G, int NW>
__device__ __forceinline__ void conv2(const u32x2* __restrict__ a1, u32x2* __restrict__ a2, const LaneWeights& w,
                                      int wave, int lane) {
    const int grp = lane >> 4, col = lane & 15;
    for (int g = wave; g * 16 < G::N2; g += NW) {
        const int p = g * 16 + col;
        const int pc = p < G::N2 ? p : G::N2 - 1;
        const int py = pc / G::AW2;
        const int base = py * G::AW1 + (pc - py * G::AW2);
        f32x4 acc = zero4();
#pragma unroll
        for (int t = 0; t < 9; ++t) acc = mfma(w.w2[t], frag(a1[(base + (t / 3) * G::AW1 + t % 3) * 4 + grp]), acc);
        if (p < G::N2)
            a2[p * 4 + grp] = pack_bf4(fmaxf(acc[0] + w.bias2[0], 0.f), fmaxf(acc[1] + w.bias2[1], 0.f),
                                       fmaxf(acc[2] + w.bias2[2], 0.f), fmaxf(acc[3] + w.bias2[3], 0.f));
    }
}

// Layer 3 at output point p of the tile (vector ALU, FP32 accumulation).
template <class G>
__device__ __forceinline__ float conv3_at(const u32x2* __restrict__ a2, const float* __restrict__ w3s, float b3,
                                          int p) {
    const int py = p / G::OW, px = p - py * G::OW;
    const u32x4* a2q = reinterpret_cast<const u32x4*>(a2);
    float y = b3;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int q = (py + t / 3) * G::AW2 + px + t % 3;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const u32x4 v = a2q[q * 2 + half];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = 8 * half + 2 * e;
                y += w3s[c * 9 + t] * bf_val(v[e] & 0xFFFFu);
                y += w3s[(c + 1) * 9 + t] * bf_val(v[e] >> 16);
            }
        }
    }
    return y;
}

// ---------------------------------------------------------------------------
// Inference over a whole grid: 32 x 32 output tiles, one per workgroup.
// ---------------------------------------------------------------------------
using InferGeo = TileGeo<32, 32>;
constexpr int kInferThreads = 256;
constexpr size_t kInferLdsBytes =
    (size_t)InferGeo::N1 * 32 +
    (size_t)(InferGeo::NXP * 8 > InferGeo::N2 * 32 ? InferGeo::NXP * 8 : InferGeo::N2 * 32) + 144 * 4;

__global__ __launch_bounds__(kInferThreads) void k_cnn_infer(const CnnPacked* __restrict__ pk,
                                                             const double* __restrict__ r,
                                                             const double* __restrict__ bvec,
                                                             double* __restrict__ x, int nx, int ny,
                                                             const double* __restrict__ r2_partials, double inv_n,
                                                             double b_scale, float c2, float c3) {
    using G = InferGeo;
    constexpr int NW = kInferThreads / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    u32x2* a1 = reinterpret_cast<u32x2*>(smem);
    u32x2* xs = a1 + G::N1 * 4;  // the input frame, later reused for A2
    u32x2* a2 = xs;
    constexpr int kUnion = (G::NXP * 8 > G::N2 * 32 ? G::NXP * 8 : G::N2 * 32) / 8;
    float* w3s = reinterpret_cast<float*>(xs + kUnion);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int oy = blockIdx.y * G::OH, ox = blockIdx.x * G::OW;
    // the residual's RMS from its norm partials (every block sums them in the same order)
    const double s = sqrt(sum_partials(r2_partials) * inv_n);
    if (!(s > 0.0)) return;  // the base guess is exact: nothing to correct
    const double inv_s = 1.0 / s;

    for (int i = tid; i < 144; i += kInferThreads) w3s[i] = pk->w3[i];
    LaneWeights w;
    load_lane_weights(pk, lane, w);
    // every global load of a thread is issued before the first conversion
    constexpr int IT = (G::NXP + kInferThreads - 1) / kInferThreads;
    double v0[IT], v1[IT];
    bool in[IT];
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        const int i = tid + t * kInferThreads;
        const int iy = i / G::XW, ix = i - iy * G::XW;
        const int gy = oy - kCnnHalo + iy, gx = ox - kCnnHalo + ix;
        in[t] = i < G::NXP && gy >= 0 && gy < ny && gx >= 0 && gx < nx;
        v0[t] = 0.0;
        v1[t] = 0.0;
        if (in[t]) {
            const int64_t idx = (int64_t)gy * nx + gx;
            v0[t] = r[idx];
            v1[t] = bvec[idx];
        }
    }
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        const int i = tid + t * kInferThreads;
        if (i < G::NXP)
            xs[i] = in[t] ? pack_bf4((float)(v0[t] * inv_s), (float)(v1[t] * b_scale), c2, c3) : u32x2{0u, 0u};
    }
    __syncthreads();
    conv1<G, NW>(xs, a1, w, wave, lane);
    __syncthreads();
    conv2<G, NW>(a1, a2, w, wave, lane);
    __syncthreads();
    const float b3 = pk->b3;
    for (int p = tid; p < G::NO; p += kInferThreads) {
        const int py = p / G::OW, px = p - py * G::OW;
        const int gy = oy + py, gx = ox + px;
        if (gy < ny && gx < nx) {
            const float y = conv3_at<G>(a2, w3s, b3, p);
            const int64_t idx = (int64_t)gy * nx + gx;
            x[idx] = x[idx] + s * (double)y;
        }
    }
}

// ---------------------------------------------------------------------------
// Training pass over crops: 16 x 16 output tiles; each workgroup takes tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... and accumulates its weight
// gradients in MFMA accumulators, written once as a per-block partial.
// ---------------------------------------------------------------------------
using TrainGeo = TileGeo<16, 16>;
constexpr int kTrainThreads = 256;

__global__ __launch_bounds__(kTrainThreads) void k_cnn_train(
    const CnnPacked* __restrict__ pk, const float* __restrict__ fields, const CropMeta* __restrict__ meta,
    const int* __restrict__ ids, int count, int crop, int mode, float* __restrict__ y_out,
    const float* __restrict__ dy_in, const float* __restrict__ e_in, float inv_npix, float* __restrict__ pgrad,
    double* __restrict__ ploss) {
    using G = TrainGeo;
    constexpr int NW = kTrainThreads / 64;
    __shared__ __align__(16) u32x2 xs[G::NXP];
    __shared__ __align__(16) u32x2 a1[G::N1 * 4];
    __shared__ __align__(16) u32x2 a2[G::N2 * 4];
    __shared__ __align__(16) u32x2 dz2[G::N2 * 4];
    __shared__ __align__(16) u32x2 dz1[G::N1 * 4];
    __shared__ float dys[G::NO];
    __shared__ float w3s[144];
    __shared__ double red_loss[NW];
    __shared__ float red_b3[NW];
    const uint16_t* xs16 = reinterpret_cast<const uint16_t*>(xs);
    const uint16_t* a1_16 = reinterpret_cast<const uint16_t*>(a1);
    const uint16_t* a2_16 = reinterpret_cast<const uint16_t*>(a2);
    const uint16_t* dz2_16 = reinterpret_cast<const uint16_t*>(dz2);
    const uint16_t* dz1_16 = reinterpret_cast<const uint16_t*>(dz1);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, col = lane & 15;
    for (int i = tid; i < 144; i += kTrainThreads) w3s[i] = pk->w3[i];
    LaneWeights w;
    load_lane_weights(pk, lane, w);
    bf16x4 w2t[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) w2t[t] = frag(reinterpret_cast<const u32x2*>(pk->w2t[t])[lane]);
    const float b3 = pk->b3;

    f32x4 gW2[9], gB2 = zero4(), gW3 = zero4(), gW1[3];
#pragma unroll
    for (int t = 0; t < 9; ++t) gW2[t] = zero4();
#pragma unroll
    for (int b = 0; b < 3; ++b) gW1[b] = zero4();
    float gb3 = 0.f;
    double lossacc = 0.0;
    const uint32_t one_bf = 0x3F80u;
    const uint32_t ones_h[4] = {one_bf, one_bf, one_bf, one_bf};
    const bf16x4 ones = frag4(ones_h);

    const int tpr = crop / 16, tpc = tpr * tpr, CP = crop + 2 * kCnnHalo;
    const int total = count * tpc;
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int j = tile / tpc, rr = tile - j * tpc;
        const int ty = rr / tpr, tx = rr - ty * tpr;
        const int id = ids[j];
        const CropMeta mt = meta[id];
        const float* f0 = fields + (int64_t)id * 2 * CP * CP;
        const float* f1 = f0 + (int64_t)CP * CP;
        __syncthreads();  // the previous tile's readers are done
        for (int i = tid; i < G::NXP; i += kTrainThreads) {
            const int iy = i / G::XW, ix = i - iy * G::XW;
            const int row = ty * 16 + iy, cl = tx * 16 + ix;
            const bool inside = row >= mt.r0 && row < mt.r1 && cl >= mt.c0 && cl < mt.c1;
            const int64_t idx = (int64_t)row * CP + cl;
            xs[i] = pack_bf4(f0[idx], f1[idx], inside ? mt.c2 : 0.f, inside ? mt.c3 : 0.f);
        }
        __syncthreads();
        conv1<G, NW>(xs, a1, w, wave, lane);
        __syncthreads();
        conv2<G, NW>(a1, a2, w, wave, lane);
        __syncthreads();
        // layer 3, loss and dL/dy
        for (int p = tid; p < G::NO; p += kTrainThreads) {
            const float y = conv3_at<G>(a2, w3s, b3, p);
            const int py = p / 16, px = p - py * 16;
            const int64_t o = (int64_t)(ty * 16 + py) * crop + tx * 16 + px;
            const int64_t q = (int64_t)j * crop * crop + o;
            if (mode == 0) {
                y_out[q] = y;
            } else {
                // dL/dy of the residual loss, formed by k_cnn_resgrad from this batch's outputs
                const float ev = e_in[q];
                lossacc += (double)ev * (double)ev;
                const float d = dy_in[q];
                dys[p] = d;
                gb3 += d;
            }
        }
        if (mode == 0) continue;
        __syncthreads();
        // dL/dz2 on the A2 frame: back through layer 3 and the ReLU
        for (int q = tid; q < G::N2; q += kTrainThreads) {
            const int qy = q / G::AW2, qx = q - qy * G::AW2;
            float da[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) da[c] = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int oy = qy - t / 3, ox = qx - t % 3;
                if (oy >= 0 && oy < 16 && ox >= 0 && ox < 16) {
                    const float d = dys[oy * 16 + ox];
#pragma unroll
                    for (int c = 0; c < 16; ++c) da[c] += w3s[c * 9 + t] * d;
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const u32x2 m = a2[q * 4 + k];
                const float v0 = bf_val(m.x & 0xFFFFu) > 0.f ? da[4 * k + 0] : 0.f;
                const float v1 = bf_val(m.x >> 16) > 0.f ? da[4 * k + 1] : 0.f;
                const float v2 = bf_val(m.y & 0xFFFFu) > 0.f ? da[4 * k + 2] : 0.f;
                const float v3 = bf_val(m.y >> 16) > 0.f ? da[4 * k + 3] : 0.f;
                dz2[q * 4 + k] = pack_bf4(v0, v1, v2, v3);
            }
        }
        __syncthreads();
        // dL/dz1 on the A1 frame: back through layer 2 (MFMA with W2^T) and the ReLU
        for (int g = wave; g * 16 < G::N1; g += NW) {
            const int p = g * 16 + col;
            const int pc = p < G::N1 ? p : G::N1 - 1;
            const int py = pc / G::AW1, px = pc - py * G::AW1;
            f32x4 acc = zero4();
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int sy = py - t / 3, sx = px - t % 3;
                const bool ok = sy >= 0 && sy < G::AH2 && sx >= 0 && sx < G::AW2;
                u32x2 v = dz2[ok ? (sy * G::AW2 + sx) * 4 + grp : 0];
                if (!ok) v = u32x2{0u, 0u};
                acc = mfma(w2t[t], frag(v), acc);
            }
            if (p < G::N1) {
                const u32x2 m = a1[p * 4 + grp];
                dz1[p * 4 + grp] = pack_bf4(bf_val(m.x & 0xFFFFu) > 0.f ? acc[0] : 0.f,
                                            bf_val(m.x >> 16) > 0.f ? acc[1] : 0.f,
                                            bf_val(m.y & 0xFFFFu) > 0.f ? acc[2] : 0.f,
                                            bf_val(m.y >> 16) > 0.f ? acc[3] : 0.f);
            }
        }
        __syncthreads();
        // weight gradients of layers 2 and 3, K = 16 points of the A2 frame per MFMA
        for (int ch = wave; ch * 16 < G::N2; ch += NW) {
            uint32_t av[4], a3[4], b3v[4];
            int base1[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = ch * 16 + 4 * grp + r;
                const bool ok = q < G::N2;
                const int qc = ok ? q : 0;
                const int qy = qc / G::AW2, qx = qc - qy * G::AW2;
                av[r] = ok ? dz2_16[qc * 16 + col] : 0u;
                b3v[r] = ok ? a2_16[qc * 16 + col] : 0u;
                base1[r] = qy * G::AW1 + qx;
                float dv = 0.f;
                if (ok && col < 9) {
                    const int oy = qy - col / 3, ox = qx - col % 3;
                    if (oy >= 0 && oy < 16 && ox >= 0 && ox < 16) dv = dys[oy * 16 + ox];
                }
                a3[r] = bf_bits(dv);
            }
            const bf16x4 A = frag4(av);
            gB2 = mfma(A, ones, gB2);
            gW3 = mfma(frag4(a3), frag4(b3v), gW3);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int off = (t / 3) * G::AW1 + t % 3;
                uint32_t bv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) bv[r] = a1_16[(base1[r] + off) * 16 + col];
                gW2[t] = mfma(A, frag4(bv), gW2[t]);
            }
        }
        // weight gradients of layer 1 (column 36 of B is 1: the bias), K = 16 points of A1
        for (int ch = wave; ch * 16 < G::N1; ch += NW) {
            uint32_t av[4];
            int basex[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = ch * 16 + 4 * grp + r;
                const bool ok = q < G::N1;
                const int qc = ok ? q : 0;
                const int qy = qc / G::AW1, qx = qc - qy * G::AW1;
                av[r] = ok ? dz1_16[qc * 16 + col] : 0u;
                basex[r] = qy * G::XW + qx;
            }
            const bf16x4 A = frag4(av);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int n = 16 * b + col;
                uint32_t bv[4];
                if (n < 36) {
                    const int tap = n >> 2, c = n & 3;
                    const int off = (tap / 3) * G::XW + tap % 3;
#pragma unroll
                    for (int r = 0; r < 4; ++r) bv[r] = xs16[(basex[r] + off) * 4 + c];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) bv[r] = (n == 36) ? one_bf : 0u;
                }
                gW1[b] = mfma(A, frag4(bv), gW1[b]);
            }
        }
    }
    if (mode == 0) return;

    // Per-block partial: waves add their accumulators in a fixed order.
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lossacc += __shfl_down(lossacc, off, 64);
        gb3 += __shfl_down(gb3, off, 64);
    }
    __syncthreads();
    if (lane == 0) {
        red_loss[wave] = lossacc;
        red_b3[wave] = gb3;
    }
    float* red = reinterpret_cast<float*>(a1);
    for (int wv = 0; wv < NW; ++wv) {
        if (wave == wv) {
            const bool first = wv == 0;
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = kOffW2 + (4 * grp + r) * 144 + col * 9 + t;
                    red[i] = first ? gW2[t][r] : red[i] + gW2[t][r];
                }
            if (col == 0)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = kOffB2 + 4 * grp + r;
                    red[i] = first ? gB2[r] : red[i] + gB2[r];
                }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = 4 * grp + r;
                if (t < 9) {
                    const int i = kOffW3 + col * 9 + t;
                    red[i] = first ? gW3[r] : red[i] + gW3[r];
                }
            }
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int n = 16 * b + col;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int o = 4 * grp + r;
                    int i = -1;
                    if (n < 36) i = kOffW1 + o * 36 + (n & 3) * 9 + (n >> 2);
                    else if (n == 36) i = kOffB1 + o;
                    if (i >= 0) red[i] = first ? gW1[b][r] : red[i] + gW1[b][r];
                }
            }
        }
        __syncthreads();
    }
    float* dst = pgrad + (int64_t)blockIdx.x * kCnnParams;
    for (int i = tid; i < kOffB3; i += kTrainThreads) dst[i] = red[i];
    if (tid == 0) {
        float sb = 0.f;
        double sl = 0.0;
        for (int wv = 0; wv < NW; ++wv) {
            sb += red_b3[wv];
            sl += red_loss[wv];
        }
        dst[kOffB3] = sb;
        ploss[blockIdx.x] = sl * (double)inv_npix;  // the loss is a mean over the batch's output points
    }
}

// Sum of the per-block partials in a fixed order (deterministic).  A workgroup
// owns 64 consecutive columns (the parameters, and the loss as column
// kCnnParams); its 16 rows of lanes each add every 16th partial with eight
// loads in flight, then one lane per column adds the 16 row sums in order.
constexpr int kRedCols = 64, kRedRows = 16;

__global__ __launch_bounds__(kRedCols * kRedRows) void k_cnn_reduce(const float* __restrict__ pgrad,
                                                                   const double* __restrict__ ploss, int nb,
                                                                   float* __restrict__ grad,
                                                                   double* __restrict__ loss) {
    __shared__ double part[kRedRows][kRedCols + 1];
    const int col = threadIdx.x % kRedCols, row = threadIdx.x / kRedCols;
    const int i = blockIdx.x * kRedCols + col;
    double s = 0.0;
    if (i < kCnnParams) {
        const float* src = pgrad + i;
        int b = row;
        for (; b + 7 * kRedRows < nb; b += 8 * kRedRows) {
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = src[(int64_t)(b + u * kRedRows) * kCnnParams];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += (double)x[u];
        }
        for (; b < nb; b += kRedRows) s += (double)src[(int64_t)b * kCnnParams];
    } else if (i == kCnnParams) {
        for (int b = row; b < nb; b += kRedRows) s += ploss[b];
    }
    part[row][col] = s;
    __syncthreads();
    if (row == 0 && i <= kCnnParams) {
        double t = 0.0;
        for (int r = 0; r < kRedRows; ++r) t += part[r][col];
        if (i < kCnnParams)
            grad[i] = (float)t;
        else
            *loss = t;
    }
}

__device__ __forceinline__ uint16_t bf_of(const float* p, int i) { return (uint16_t)bf_bits(p[i]); }

// Adam update (optional) then the parameter image; one workgroup.
__global__ __launch_bounds__(1024) void k_cnn_adam_pack(float* __restrict__ params, float* __restrict__ m,
                                                        float* __restrict__ v, const float* __restrict__ grad,
                                                        float lr, float beta1, float beta2, float eps, float inv_c1,
                                                        float inv_c2, int do_adam, CnnPacked* __restrict__ pk) {
    const int tid = threadIdx.x;
    if (do_adam) {
        for (int i = tid; i < kCnnParams; i += 1024) {
            const float g = grad[i];
            const float mi = beta1 * m[i] + (1.f - beta1) * g;
            const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
            m[i] = mi;
            v[i] = vi;
            params[i] -= lr * (mi * inv_c1) / (sqrtf(vi * inv_c2) + eps);
        }
    }
    __syncthreads();
    for (int e = tid; e < 3 * 64 * 4; e += 1024) {
        const int t = e / 256, lane = (e / 4) % 64, r = e % 4;
        const int o = lane & 15, tap = 4 * t + (lane >> 4), c = r;
        pk->w1[t][lane][r] = tap < 9 ? bf_of(params, kOffW1 + o * 36 + c * 9 + tap) : (uint16_t)0;
    }
    for (int e = tid; e < 9 * 64 * 4; e += 1024) {
        const int t = e / 256, lane = (e / 4) % 64, r = e % 4;
        const int row = lane & 15, k = 4 * (lane >> 4) + r;
        pk->w2[t][lane][r] = bf_of(params, kOffW2 + row * 144 + k * 9 + t);   // A[o = row][c = k]
        pk->w2t[t][lane][r] = bf_of(params, kOffW2 + k * 144 + row * 9 + t);  // A[c = row][o = k]
    }
    if (tid < 16) {
        pk->b1[tid] = params[kOffB1 + tid];
        pk->b2[tid] = params[kOffB2 + tid];
    }
    if (tid < 144) pk->w3[tid] = bf_val(bf_bits(params[kOffW3 + tid]));
    if (tid == 0) pk->b3 = params[kOffB3];
}

__global__ __launch_bounds__(256) void k_cnn_extract(const double* __restrict__ r, const double* __restrict__ bvec,
                                                     int nx, int ny, double inv_s, double b_scale,
                                                     const int* __restrict__ origins, int crop,
                                                     float* __restrict__ fields_out, float* __restrict__ target_out) {
    const int j = blockIdx.y;
    const int oy = origins[2 * j], ox = origins[2 * j + 1];
    const int CP = crop + 2 * kCnnHalo;
    float* f0 = fields_out + (int64_t)j * 2 * CP * CP;
    float* f1 = f0 + (int64_t)CP * CP;
    float* tg = target_out + (int64_t)j * crop * crop;
    const int stride = gridDim.x * 256;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < CP * CP; i += stride) {
        const int iy = i / CP, ix = i - iy * CP;
        const int gy = oy - kCnnHalo + iy, gx = ox - kCnnHalo + ix;
        float v0 = 0.f, v1 = 0.f;
        if (gy >= 0 && gy < ny && gx >= 0 && gx < nx) {
            const int64_t idx = (int64_t)gy * nx + gx;
            v0 = (float)(r[idx] * inv_s);
            v1 = (float)(bvec[idx] * b_scale);
        }
        f0[i] = v0;
        f1[i] = v1;
    }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < crop * crop; i += stride) {
        const int iy = i / crop, ix = i - iy * crop;
        const int64_t idx = (int64_t)(oy + iy) * nx + (ox + ix);
        tg[i] = (float)(r[idx] * inv_s);
    }
}

// ---------------------------------------------------------------------------
// Residual loss of the residual form on one batch of crops.  M = I - a L_h in
// units of the spacing (ahx = a / h_x^2, ahy = a / h_y^2); values beyond a
// window edge that lies on a wall follow the wall closure of L_h (the wall
// value 0, and for order 4 the odd-reflection ghost), values beyond any other
// edge are never read for e (its loss points keep the stencil inside the
// window) and read as 0 for dy (e is 0 outside the window).
// ---------------------------------------------------------------------------
struct CropEdges {
    bool top, bot, left, right;  // window edges on a wall of the grid
};

__device__ __forceinline__ CropEdges crop_edges(const CropMeta& m, int crop) {
    CropEdges e;
    e.top = m.r0 == kCnnHalo;
    e.bot = m.r1 == kCnnHalo + crop;
    e.left = m.c0 == kCnnHalo;
    e.right = m.c1 == kCnnHalo + crop;
    return e;
}

// Value of window function f at (row, col), one or two cells beyond the
// window included: beyond a wall edge the closure, beyond any other edge 0.
__device__ __forceinline__ float crop_at(const float* f, int crop, const CropEdges& ed, int row, int col) {
    if (row < 0) {
        if (!ed.top || row == -1) return 0.f;
        return -f[(int64_t)0 * crop + col];          // ghost -u_0 two cells beyond the wall
    }
    if (row >= crop) {
        if (!ed.bot || row == crop) return 0.f;
        return -f[(int64_t)(crop - 1) * crop + col];
    }
    if (col < 0) {
        if (!ed.left || col == -1) return 0.f;
        return -f[(int64_t)row * crop + 0];
    }
    if (col >= crop) {
        if (!ed.right || col == crop) return 0.f;
        return -f[(int64_t)row * crop + crop - 1];
    }
    return f[(int64_t)row * crop + col];
}

// (M f)(row, col) on the window with the closures of crop_at.
__device__ __forceinline__ float crop_M_at(const float* f, int crop, const CropEdges& ed, const CropMeta& m, int row,
                                           int col) {
    const float c = f[(int64_t)row * crop + col];
    float dx, dy;
    if (m.order == 2) {
        dx = crop_at(f, crop, ed, row, col - 1) + crop_at(f, crop, ed, row, col + 1) - 2.f * c;
        dy = crop_at(f, crop, ed, row - 1, col) + crop_at(f, crop, ed, row + 1, col) - 2.f * c;
    } else {
        dx = (16.f * (crop_at(f, crop, ed, row, col - 1) + crop_at(f, crop, ed, row, col + 1)) -
              (crop_at(f, crop, ed, row, col - 2) + crop_at(f, crop, ed, row, col + 2)) - 30.f * c) *
             (1.f / 12.f);
        dy = (16.f * (crop_at(f, crop, ed, row - 1, col) + crop_at(f, crop, ed, row + 1, col)) -
              (crop_at(f, crop, ed, row - 2, col) + crop_at(f, crop, ed, row + 2, col)) - 30.f * c) *
             (1.f / 12.f);
    }
    return c - (m.ahx * dx + m.ahy * dy);
}

__global__ __launch_bounds__(256) void k_cnn_resid(const float* __restrict__ y, const float* __restrict__ target,
                                                   const CropMeta* __restrict__ meta, const int* __restrict__ ids,
                                                   int crop, float* __restrict__ e_out) {
    const int j = blockIdx.y;
    const int id = ids[j];
    const CropMeta m = meta[id];
    const CropEdges ed = crop_edges(m, crop);
    const int R = m.order / 2;
    const float* yj = y + (int64_t)j * crop * crop;
    const float* tj = target + (int64_t)id * crop * crop;
    float* ej = e_out + (int64_t)j * crop * crop;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < crop * crop; i += gridDim.x * 256) {
        const int row = i / crop, col = i - row * crop;
        const bool ok = (row >= R || ed.top) && (row <= crop - 1 - R || ed.bot) && (col >= R || ed.left) &&
                        (col <= crop - 1 - R || ed.right);
        ej[i] = ok ? tj[i] - crop_M_at(yj, crop, ed, m, row, col) : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_cnn_resgrad(const float* __restrict__ e, const CropMeta* __restrict__ meta,
                                                     const int* __restrict__ ids, int crop, float scale,
                                                     float* __restrict__ dy_out) {
    const int j = blockIdx.y;
    const CropMeta m = meta[ids[j]];
    const CropEdges ed = crop_edges(m, crop);
    const float* ej = e + (int64_t)j * crop * crop;
    float* dj = dy_out + (int64_t)j * crop * crop;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < crop * crop; i += gridDim.x * 256) {
        const int row = i / crop, col = i - row * crop;
        dj[i] = scale * crop_M_at(ej, crop, ed, m, row, col);
    }
}

}  // namespace

hipError_t launch_cnn_pack(const float* params, CnnPacked* pk, hipStream_t s) {
    k_cnn_adam_pack<<<1, 1024, 0, s>>>(const_cast<float*>(params), nullptr, nullptr, nullptr, 0.f, 0.f, 0.f, 0.f,
                                       0.f, 0.f, 0, pk);
    return hipGetLastError();
}

hipError_t launch_cnn_adam_pack(float* params, float* m, float* v, const float* grad, float lr, float beta1,
                                float beta2, float eps, float inv_c1, float inv_c2, CnnPacked* pk, hipStream_t s) {
    k_cnn_adam_pack<<<1, 1024, 0, s>>>(params, m, v, grad, lr, beta1, beta2, eps, inv_c1, inv_c2, 1, pk);
    return hipGetLastError();
}

hipError_t launch_cnn_infer(const CnnPacked* pk, const double* r, const double* b, double* x, int nx, int ny,
                            const double* r2_partials, double inv_n, double b_scale, float c2, float c3,
                            hipStream_t st) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_cnn_infer, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)kInferLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    dim3 grid((unsigned)((nx + InferGeo::OW - 1) / InferGeo::OW), (unsigned)((ny + InferGeo::OH - 1) / InferGeo::OH));
    k_cnn_infer<<<grid, kInferThreads, kInferLdsBytes, st>>>(pk, r, b, x, nx, ny, r2_partials, inv_n, b_scale, c2,
                                                             c3);
    return hipGetLastError();
}

hipError_t launch_cnn_extract(const double* r, const double* b, int nx, int ny, double inv_s, double b_scale,
                              const int* origins_dev, int ncrop, int crop, float* fields_out, float* target_out,
                              hipStream_t st) {
    if (ncrop <= 0) return hipSuccess;
    dim3 grid(16u, (unsigned)ncrop);
    k_cnn_extract<<<grid, 256, 0, st>>>(r, b, nx, ny, inv_s, b_scale, origins_dev, crop, fields_out, target_out);
    return hipGetLastError();
}

hipError_t launch_cnn_resloss(const float* y, const float* target, const CropMeta* meta, const int* ids, int count,
                              int crop, float inv_npix, float* e_out, float* dy_out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    dim3 grid(16u, (unsigned)count);
    k_cnn_resid<<<grid, 256, 0, st>>>(y, target, meta, ids, crop, e_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_cnn_resgrad<<<grid, 256, 0, st>>>(e_out, meta, ids, crop, -2.f * inv_npix, dy_out);
    return hipGetLastError();
}

int cnn_train_blocks(int count, int crop) {
    const int tiles = count * (crop / 16) * (crop / 16);
    return tiles < kCnnTrainBlocks ? tiles : kCnnTrainBlocks;
}

hipError_t launch_cnn_train(const CnnPacked* pk, const float* fields, const CropMeta* meta, const int* ids,
                            int count, int crop, int mode, float* y_out, const float* dy_in, const float* e_in,
                            float inv_npix, float* pgrad, double* ploss, int nblocks, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    k_cnn_train<<<nblocks, kTrainThreads, 0, st>>>(pk, fields, meta, ids, count, crop, mode, y_out, dy_in, e_in,
                                                   inv_npix, pgrad, ploss);
    return hipGetLastError();
}

hipError_t launch_cnn_reduce(const float* pgrad, const double* ploss, int nblocks, float* grad, double* loss,
                             hipStream_t st) {
    k_cnn_reduce<<<(kCnnParams + kRedCols) / kRedCols, kRedCols * kRedRows, 0, st>>>(pgrad, ploss, nblocks, grad, loss);
    return hipGetLastError();
}

}  // namespace ew

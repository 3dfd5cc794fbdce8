// Declarations shared by the batched form (batch.hip, batch_kernels.hip).
#pragma once

#include "ew_internal.h"

namespace ew {

constexpr int kBatchSmallThreads = 1024;
constexpr int kBatchSmallPts = 16;       // points per thread: small problems have <= 16384 points
constexpr int kBatchSmallMaxSide = 128;  // and nx, ny <= 128 (LDS (nx+4)(ny+4) floats <= 70 KB)
constexpr int kConvPerThread = 8;

// Per-problem state visible to the kernels (device array, refreshed before
// every batched wave-solve).
// The state arrays hold the batch's state type T (float for FP32 state,
// double for FP64 state); with FP64 state f0 is the caller's v and acc its
// out, set before every batched wave-solve.
struct BatchProbDev {
    Geo g;
    int order;
    int n_t;
    int coef_off;
    int active;
    double dt2;
    const double* v;   // W^0 (FP64, caller's vector)
    double* out;       // S v (FP64)
    void* f0;          // W^0 in the state type
    void* fA;          // odd time levels (FP64 state: the latest level after an even launch)
    void* fB;          // even time levels >= 2 (FP64 state: the level before it)
    void* fC;          // FP64 state: the latest level after an odd launch
    void* fD;          // FP64 state: the level before it
    void* acc;         // filter accumulator
};

// Per-problem description of one batched Gram-Schmidt chain.
struct BatchMgsDev {
    double* w;
    int64_t n;
    int q;         // chain length: number of basis vectors + 1 (0 = problem idle this step)
    int nblk;      // reduction blocks of this problem
    int part_off;  // offset of its two partial-sum arrays
    int h_off;     // offset of its coefficients in the output
};

struct MgsLink {
    const double* u;
};

// One workgroup of a batched step launch: the problem it advances and the
// tile of that problem, so that a workgroup finds both with one load.
struct BatchBlk {
    int prob;
    int tile;
};

hipError_t launch_batch_small(BatchProbDev* probs, const int* small_ids, int nsmall, const float* coef, int order,
                              size_t lds_bytes, hipStream_t s);
hipError_t prepare_batch_small(int order, size_t lds_bytes);
// coef: float (FP32 state) or double (fp64 != 0) filter weights.
// blk: nblocks entries (problems ordered so that the ones still stepping at
// `step` are covered by the first nblocks workgroups).
hipError_t launch_batch_step(BatchProbDev* probs, const BatchBlk* blk, int nblocks, const void* coef, int step,
                             int order, int tyr, int fp64, hipStream_t s);
// FP64 state: steps L S .. L S + S - 1 of every problem in launch L (S =
// batch_steps_per_launch(order); a problem with fewer steps left does those),
// in 16 x 16 tiles with 8-point halos (batch_blocked_tiles per problem; blk
// as for launch_batch_step, the first nblocks workgroups covering the
// problems still stepping at step L S).  Launch 0 reads W^0 from f0; launch
// L > 0 reads the two levels launch L - 1 wrote, and launch L writes its last
// two levels to (fA, fB) for even L and to (fC, fD) for odd L.
int batch_steps_per_launch(int order);
int batch_blocked_tiles(const Geo& g);
hipError_t launch_batch_blocked(BatchProbDev* probs, const BatchBlk* blk, int nblocks, const double* coef, int launch,
                                int order, hipStream_t s);
hipError_t launch_batch_convert(BatchProbDev* probs, const int* ids, const int* blk_start, int nseg, int nblocks,
                                int to_fp32, hipStream_t s);
hipError_t launch_batch_mgs(const BatchMgsDev* info, const MgsLink* links, int nprob, const int* blk_start,
                            int nblocks, int ell, double* partial, double* hout, hipStream_t s);

}  // namespace ew

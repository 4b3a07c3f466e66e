// mlp.hpp -- learned velocity surrogate: sizes, parameter layout and the
// launchers of the training kernels (internal).
//
// Network 193 -> 128 -> 128 -> 128 -> 3, tanh-GELU after the hidden layers.
// FP32 master parameters in one flat vector, layer by layer: W_l as [fan_in][fan_out]
// (row-major), then b_l.  The matrix-core kernels read BF16 copies of the weights:
//   wt[l]  W_l^T as [MP_l][KP_l]  (fan-out rows padded to 16, fan-in to 32)
//   wn[l]  W_l   as [KP_l][CP_l]  (fan-out padded to a 32-wide contraction),
//          layers 2-4 only (the backward product needs no input gradient of layer 1).
//   wtp[l], wnp[l]  the same as wt[l], wn[l] for layers 2-4 with each row in the
//          permuted slot order of the training pass (column 32q + 16s + 4g + j
//          stored at 32q + 8g + 4s + j), so that a product fragment is one
//          16-byte load.
// Padding entries are zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpl {
namespace mlp {

constexpr int kFeat = 193;   // raw features
constexpr int kHid = 128;
constexpr int kOut = 3;
constexpr int kLayers = 4;

__host__ __device__ constexpr int fan_in(int l) { return l == 0 ? kFeat : kHid; }
__host__ __device__ constexpr int fan_out(int l) { return l == 3 ? kOut : kHid; }
__host__ __device__ constexpr int kpad(int l) { return l == 0 ? 224 : kHid; }   // multiple of 32
__host__ __device__ constexpr int mpad(int l) { return l == 3 ? 16 : kHid; }    // multiple of 16
__host__ __device__ constexpr int cpad(int l) { return l == 3 ? 32 : kHid; }    // multiple of 32
__host__ __device__ constexpr int64_t off_w(int l) {
    return l == 0 ? 0 : off_w(l - 1) + (int64_t)fan_in(l - 1) * fan_out(l - 1) + fan_out(l - 1);
}
__host__ __device__ constexpr int64_t off_b(int l) { return off_w(l) + (int64_t)fan_in(l) * fan_out(l); }
constexpr int64_t kNParam = off_b(3) + kOut;
static_assert(kNParam == 58243, "parameter count");
// Position of column c of a row in the permuted slot order.
__host__ __device__ constexpr int perm_col(int c) {
    return (c & ~31) | (((c >> 2) & 3) << 3) | (((c >> 4) & 1) << 2) | (c & 3);
}
constexpr int kK1 = 224;     // padded layer-1 fan-in (and the length of mean/1/std)

// Training and batch-inference buffers, sized for max_batch rows.
struct TrainBufs {
    int64_t max_batch = 0;
    uint16_t *x0 = nullptr;                        // standardised input [B][224] (batch inference)
    uint16_t *h[3] = {};                           // hidden activations [B][128] (batch inference)
    float *y = nullptr;                            // output [B][16] (batch inference)
    uint16_t *tr = nullptr;                        // training: BF16 transposed rows, blocked (below)
    float *part_w[4] = {};                         // per-chunk weight gradients [nchunk][MP][KP]
    double *part_b[4] = {};                        // per-workgroup bias gradients [ngroup][MP]
    double *loss_part = nullptr;                   // per-16-row tile [B/16]
    float *grads = nullptr;                        // [kNParam]
};

// Rows of the training pass's transposed output: the layer-1 input (224
// rows), the hidden activations of layers 1-3 (3 x 128), the output gradients
// of layers 1-3 (3 x 128) and of layer 4 (16).  Stored in blocks of kTrBlock
// batch rows, element (row r, batch row b) at
// tr[(b / kTrBlock) kTrRows kTrBlock + r kTrBlock + b % kTrBlock], so that a
// workgroup of the pass writes one contiguous block.
constexpr int kTrHt = kK1, kTrDz = kK1 + 3 * kHid, kTrRows = kTrDz + 3 * kHid + 16;
constexpr int kTrBlock = 32;

constexpr int64_t kChunk = 256;   // rows per workgroup in the weight-gradient products
inline int64_t n_chunks(int64_t B) { return (B + kChunk - 1) / kChunk; }
constexpr int64_t kTrainGroupRows = kTrBlock;   // rows per workgroup of the training pass
inline int64_t n_train_groups(int64_t B) { return (B + kTrainGroupRows - 1) / kTrainGroupRows; }

// Device state of one network (owned by the couple_mlp handle).
struct NetBufs {
    float *params = nullptr, *m = nullptr, *v = nullptr;   // FP32 master and Adam moments [kNParam]
    uint16_t *wt[4] = {}, *wn[4] = {};
    uint16_t *wtp[4] = {}, *wnp[4] = {};                    // permuted copies, layers 2-4
    float *mean_inv = nullptr;                              // [2][224]
};

// Kernel launchers (mlp.hip).  All enqueue on `st` and return the launch status.
hipError_t launch_cast(const NetBufs &net, hipStream_t st);
// Batch inference: standardise B rows of feat into x0, then the four layers into y.
hipError_t launch_standardise(const float *feat, int64_t B, const float *mean_inv, uint16_t *x0, hipStream_t st);
hipError_t launch_forward(const NetBufs &net, const TrainBufs &tb, int64_t B, hipStream_t st);
// Gradient of the mean loss over a batch of B rows (a multiple of 32): rows
// idx[b] (or b) of feat [nrows][193] and resid [nrows][3]; grads [kNParam] and
// (if loss) the loss.
hipError_t launch_gradients(const NetBufs &net, const TrainBufs &tb, const float *feat, const float *resid,
                            const int32_t *idx, int64_t nrows, int64_t B, const float inv_scale[3], float *grads,
                            float *loss, hipStream_t st);
// b1, b2 and their complements 1 - b1, 1 - b2 are rounded separately from
// double (0.999f alone would leave 1 - b2 off by 1e-5 relative).
hipError_t launch_adam(const NetBufs &net, const float *grads, float lr, float b1, float omb1, float b2, float omb2,
                       float eps, float c1, float c2, hipStream_t st);
hipError_t launch_output(const TrainBufs &tb, int64_t B, float *y, hipStream_t st);
// Per-column mean and population standard deviation (two passes, FP64, fixed
// order) of a row-major [n][cols] matrix, cols <= 256; part holds nchunk * cols.
hipError_t launch_column_stats(const float *x, int64_t n, int cols, double *part, int64_t nchunk, double *mean,
                               double *std, hipStream_t st);
hipError_t launch_features(const int nb[3], const double box[3], int64_t n, const float *pos, const float *diam,
                           const float *phi, const float *U, const float *G, const float *u_fine,
                           const int32_t *sel, int64_t nsel, float *feat, float *u_bulk, float *resid,
                           hipStream_t st);

}  // namespace mlp
}  // namespace cpl

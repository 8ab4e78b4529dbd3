// Host-side planning shared by the C ABI: workspace layout and launch sequences.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "msibm.h"

namespace msibm {

int level_dim(int v, int k);
int level_range(int D, int k);
int auto_levels(int D);
size_t align_up(size_t v);

// Window half-width n_k of level k: the per-level entry, or the common one.
inline int level_n(const msibm_config* cfg, int k)
{
    const int v = (k >= 0 && k < MSIBM_MAX_LEVELS) ? cfg->half_window_levels[k] : 0;
    return v ? v : cfg->half_window;
}

// Workspace offsets of one pair.  Level k (k >= 1) holds both views' pyramid
// images (float, W_k pitch); every level holds both views' window statistics
// (12 bytes per pixel); levels k >= 1 hold the winner-take-all map (int16).
struct PairLayout {
    int K;
    int h[MSIBM_MAX_LEVELS], w[MSIBM_MAX_LEVELS];
    size_t img[MSIBM_MAX_LEVELS][2];
    size_t stat[MSIBM_MAX_LEVELS][2];
    size_t map[MSIBM_MAX_LEVELS];
    size_t blur[2];           // pre-blurred level 0 (float, pitch W), when asked for
    size_t cmap[MSIBM_MAX_LEVELS]; // levels k >= 1: the cost map (float), with the gating
    size_t dtmp;              // unfiltered map of a level (int16), with the median
    size_t ctmp;              // level 0's cost (float) when the caller takes none
    size_t grad[MSIBM_MAX_LEVELS][2]; // levels 1..K-2: both views' image gradients (float),
                                      // for the backward through every level
    size_t l1acc;             // the fused masked-L1 step: {int |M|, float sum |d_soft - gt|}
    size_t bytes;
};

PairLayout pair_layout(const msibm_pair& p, int K, bool preblur = false, bool median = false,
                       bool gated = false, bool level_grads = false);

// Forward with a soft output at every level below the coarsest.
int run_pair_levels(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                    float* const* soft, int16_t* const* maps, hipStream_t s, std::string* err);

// Backward of a loss on every level's soft output down to the level-0 images.
int run_pair_backward_levels(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                             const int16_t* const* maps, const float* const* grad_soft, float* grad_left,
                             float* grad_right, hipStream_t s, std::string* err);

struct BatchOutputs {
    int16_t* const* disp;
    float* const* cost;
    float* const* soft;
    int16_t* const* prior1;
};

// Plain per-pair forward: 2K launches on `s`.  Levels below lowest_level are
// not matched (their pyramid images and statistics are still built).
int run_pair_plain(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                   int16_t* disp, float* cost, float* soft, int16_t* prior1, hipStream_t s,
                   std::string* err, int lowest_level = 0);

// Buffers of the fused forward, masked-L1 loss and backward of one pair.
struct FusedL1Pair {
    const float* gt;          // ground-truth disparity, H x W, pitch W
    const uint8_t* mask;      // loss pixels (nonzero), H x W, pitch W
    int16_t* disp;            // level-0 hard winner over the soft interval
    float* cost;              // its score, or NULL
    float* soft;              // level-0 d_soft
    int16_t* prior1;          // level-1 map, or NULL (then kept in the workspace)
    float* grad_left;
    float* grad_right;
    float* loss;              // one float
};

// Levels K-1..1 of the forward, then one fused launch for level 0: its soft
// level, the masked-L1 gradient and the backward to both images.
int run_pair_fused_l1(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                      const FusedL1Pair& io, hipStream_t s, std::string* err);

// The same for several pairs, stage by stage (optionally replayed from a graph).
int run_batched_fused_l1(const msibm_pair* pairs, int n_pairs, const msibm_config* cfg, const FusedL1Pair* io,
                         void* workspace, size_t ws_bytes, hipStream_t s, std::string* err);

int run_pair_backward(const msibm_pair& P, const PairLayout& lay, const msibm_config* cfg, char* ws,
                      const int16_t* prior1, const float* grad_soft, float* grad_left,
                      float* grad_right, hipStream_t s, std::string* err);

size_t batch_extra_bytes(const msibm_pair* pairs, int n_pairs, const msibm_config* cfg);

int run_batched(const msibm_pair* pairs, int n_pairs, const msibm_config* cfg, const BatchOutputs& out,
                void* workspace, size_t ws_bytes, hipStream_t s, std::string* err);

struct BatchGrads {
    const int16_t* const* prior1;
    const float* const* grad_soft;
    float* const* grad_left;
    float* const* grad_right;
};

// Batched backward: one statistics, one zero and one backward launch for all pairs.
int run_batched_backward(const msibm_pair* pairs, int n_pairs, const msibm_config* cfg, const BatchGrads& g,
                         void* workspace, size_t ws_bytes, hipStream_t s, std::string* err);

}  // namespace msibm

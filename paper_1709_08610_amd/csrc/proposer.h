// Learned seed proposer: internal interface between the host code and the
// proposer kernels.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rt {

struct Desc;

constexpr int kImg = 128;                 // slope-image side (bins)
constexpr int kPix = kImg * kImg;
constexpr int kLayers = 4;
constexpr int kChan[kLayers + 1] = {2, 64, 128, 96, 1};
constexpr float kSlopeLo = -0.35f;        // image range in both slopes
constexpr float kSlopeHi = 0.35f;

// padded K (= 9 * Cin rounded up to the GEMM K tile) of a layer's weights
__host__ __device__ constexpr int conv_k(int cin) { return 9 * cin; }
__host__ __device__ constexpr int conv_kp(int cin) { return (9 * cin + 31) / 32 * 32; }

struct NetLayout {
    int64_t w_off[kLayers];   // offset of W[l] (COUT x Kp, row-major) in the flat parameter array
    int64_t b_off[kLayers];   // offset of b[l]
    int64_t total;            // padded parameter count
    int64_t logical;          // 186,625 = sum of 9 Cin Cout + Cout
};
NetLayout net_layout();

enum GemmMode { kFwd = 0, kBwdData = 1, kBwdW = 2 };

// One implicit-GEMM launch (see proposer.hip for the index maps).
struct GemmArgs {
    int mode;
    int B;                     // images
    int cin, cout;             // channels of the layer (input, output)
    int act;                   // kFwd epilogue: 0 none (store FP32 logits), 1 ReLU (store BF16)
    const uint16_t* x;         // kFwd/kBwdW: layer input (B, H, W, cin) bf16
    const uint16_t* w;         // kFwd: W (cout, Kp) bf16; kBwdData: Wt (cin, Kpt) bf16
    const float* bias;         // kFwd
    const uint16_t* dz;        // kBwdData/kBwdW: grad wrt the layer's pre-activation (B, H, W, cout) bf16
    const uint16_t* xprev;     // kBwdData: layer input again (ReLU mask of the previous layer), or NULL
    uint16_t* y_bf16;          // kFwd act=1 output; kBwdData output (grad wrt previous pre-activation)
    float* y_f32;              // kFwd act=0 output (logits)
    float* partial;            // kBwdW: (n_chunks, cout, Kp) fp32
    int pix_per_chunk;         // kBwdW: pixels reduced by one work-group column
};
void launch_gemm(const GemmArgs& a, hipStream_t st);

// forward pass of the four layers (direct convolutions; see proposer.hip).
// train: store act1..act3 for the backward pass; otherwise only act2 and the
// head's band-edge terms u (head_edge_floats(E) floats) pass through HBM.
int prepare_forward();
size_t head_edge_floats(int64_t n_events);
void launch_forward(const uint16_t* img, const uint16_t* wbf, const float* w32, const NetLayout& L, int64_t E,
                    uint16_t* act1, uint16_t* act2, uint16_t* act3, float* u, float* logits, bool train,
                    hipStream_t st);

void launch_bin_image(const float* hits, const int32_t* plane_off, int n_planes, int meas_dim,
                      const float* plane_z, int64_t n_events, uint16_t* img, const uint32_t* err, hipStream_t st);
void launch_target_image(const double* targets, const int64_t* target_off, int64_t n_events,
                         uint8_t* tgt, hipStream_t st);
void launch_bce(const float* logits, const uint8_t* tgt, int64_t n, float pos_weight, float* loss_part,
                uint16_t* dz, hipStream_t st);
void launch_transpose_w(const uint16_t* w, int cin, int cout, uint16_t* wt, hipStream_t st);
void launch_reduce_dw(const float* partial, int n_chunks, int64_t n, float* grad, hipStream_t st);
void launch_bias_grad(const uint16_t* dz, int64_t n_pix, int cout, int n_chunks, float* partial,
                      float* grad_b, hipStream_t st);
void launch_adam(float* w, float* m, float* v, const float* g, uint16_t* wbf, int64_t n, float lr,
                 float b1, float b2, float eps, int64_t step, hipStream_t st);
void launch_to_bf16(const float* w, uint16_t* wbf, int64_t n, hipStream_t st);
void launch_sum(const float* part, int n, float* out, hipStream_t st);

// seeds from the heatmap (logits): bins above tau (local maxima with nms),
// best k_max per event; events whose best score is below conf_min fall back to the lattice
struct ProposeArgs {
    const float* logits;       // (E, kPix)
    int64_t n_events;
    int k_max;
    float ltau;                // logit(tau): candidate threshold
    float lconf;               // logit(conf_min): events whose best logit is below fall back
    int nms;                   // 1: strict 3x3 local maxima only
    int lattice_n[2];
    const float* lat_coord;    // fallback lattice cell centres (device; dimension 0 then 1)
    float bin_centre[kImg];    // slope at the centre of each image bin, formed on the host
    float* cand_score;         // scratch (E, k_max)
    int32_t* cand_pix;         // scratch (E, k_max)
    int32_t* count;            // (E) seeds of the event
    float* confidence;         // (E) best heatmap value
    int32_t* fallback;         // (E) 1: lattice seeds
    int64_t* seed_off;         // (E + 1) output offsets
    double* seeds;             // output, 4 per seed (x0, y0, tx, ty)
};
void launch_propose_select(const ProposeArgs& a, hipStream_t st);
void launch_propose_offsets(const ProposeArgs& a, hipStream_t st);
void launch_propose_write(const ProposeArgs& a, hipStream_t st);
void launch_flag_fallback(int32_t* ev_flags, const int32_t* fallback, int64_t n_events, hipStream_t st);
void launch_flag_fallback_desc(const Desc* d, const int32_t* fallback, int64_t n_events, hipStream_t st);

}  // namespace rt

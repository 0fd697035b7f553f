// Learned seed proposer kernels (gfx950).
//
// A four-layer 3x3 convolutional network (2 -> 64 -> 128 -> 96 -> 1 channels,
// ReLU between layers, a sigmoid heatmap at the end) maps an event's binned
// slope image (x/z, y/z) to a heatmap of likely track slopes.  All three
// convolution products (forward, backward to the input, backward to the
// weights) run through one implicit-GEMM kernel on BF16 MFMA with FP32
// accumulation; activations and gradients are stored in BF16, weights keep an
// FP32 master copy updated by Adam.
//
// Layout: images NHWC (batch, row = tx bin, column = ty bin, channel), channel
// fastest.  Weights W[co][tap * Cin + ci] with tap = 3 * (dr + 1) + (dc + 1),
// rows padded with zeros to a multiple of 32 (the GEMM K tile).
#include "proposer.h"
#include "rt_internal.h"

namespace rt {

typedef short v4s __attribute__((ext_vector_type(4)));
// 16-byte staging registers: a native vector (HIP's uint4 struct is copied
// through memory, which keeps staged values out of registers)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

NetLayout net_layout()
{
    NetLayout L;
    int64_t off = 0, logical = 0;
    for (int l = 0; l < kLayers; ++l) {
        const int cin = kChan[l], cout = kChan[l + 1];
        L.w_off[l] = off;
        off += (int64_t)cout * conv_kp(cin);
        L.b_off[l] = off;
        off += cout;
        logical += (int64_t)cout * conv_k(cin) + cout;
    }
    L.total = off;
    L.logical = logical;
    return L;
}

// ------------------------------------------------------------------ binning
// One work-group per event: a 2 x 128 x 128 histogram of hit slopes (x/z,
// y/z) in LDS, channel 0 for the first half of the planes, 1 for the second;
// written as log1p(count) in BF16.  Events of at most 65,535 hits keep both
// channels' counts as 16-bit halves of one word (no count can overflow);
// larger events take one pass per channel with 32-bit counts.
__device__ __forceinline__ int slope_bin(float x, float y, float z, float w)
{
    const float u = (x / z - kSlopeLo) / w;
    const float v = (y / z - kSlopeLo) / w;
    if (u >= 0.0f && u < (float)kImg && v >= 0.0f && v < (float)kImg) return (int)u * kImg + (int)v;
    return -1;
}

// err (may be NULL): validation bits of the staging that produced plane_off;
// non-zero leaves the image unwritten (the offsets may then be stale)
__global__ __launch_bounds__(256) void k_bin_image(const float* __restrict__ hits,
                                                   const int32_t* __restrict__ plane_off, int P, int D,
                                                   const float* __restrict__ plane_z, int64_t E,
                                                   uint16_t* __restrict__ img, const uint32_t* __restrict__ err)
{
    __shared__ __attribute__((aligned(16))) uint32_t s_h[kPix];  // read and cleared as uint4
    __shared__ int s_po[kMaxPlanes + 1];
    __shared__ float s_z[kMaxPlanes];
    __shared__ uint16_t s_lut[256];  // BF16(log1p(n)) for the common small counts
    if (err && *err) return;
    const float w = (kSlopeHi - kSlopeLo) / kImg;
    for (int n = threadIdx.x; n < 256; n += blockDim.x) s_lut[n] = f2bf(log1pf((float)n));
    auto enc = [&](uint32_t n) -> uint32_t { return n < 256 ? s_lut[n] : f2bf(log1pf((float)n)); };
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int32_t* po = plane_off + e * (P + 1);
        if ((int)threadIdx.x <= P) s_po[threadIdx.x] = po[threadIdx.x];
        if ((int)threadIdx.x < P) s_z[threadIdx.x] = plane_z[threadIdx.x];
        for (int i = threadIdx.x; i < kPix / 4; i += blockDim.x) reinterpret_cast<uint4*>(s_h)[i] = make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();
        const int h0 = s_po[0], h1 = s_po[P];
        const bool packed = h1 - h0 <= 0xFFFF;
        for (int pass = 0; pass < (packed ? 1 : 2); ++pass) {
            if (pass) {
                for (int i = threadIdx.x; i < kPix / 4; i += blockDim.x)
                    reinterpret_cast<uint4*>(s_h)[i] = make_uint4(0u, 0u, 0u, 0u);
                __syncthreads();
            }
            // one walk over the event's hits (sorted by plane): a hit's plane is
            // the last p with s_po[p] <= k, found by bisection
            for (int k = h0 + threadIdx.x; k < h1; k += blockDim.x) {
                int lo = 0, hi = P;  // s_po[lo] <= k < s_po[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_po[mid] <= k) lo = mid;
                    else hi = mid;
                }
                const int ch = lo < P / 2 ? 0 : 1;
                if (!packed && ch != pass) continue;
                const float x = hits[(int64_t)k * D];
                const float y = D == 2 ? hits[(int64_t)k * D + 1] : 0.0f;
                const int bin = slope_bin(x, y, s_z[lo], w);
                if (bin >= 0) atomicAdd(&s_h[bin], packed ? 1u << (16 * ch) : 1u);
            }
            __syncthreads();
            if (packed) {
                // four pixels (both channels each) per 16-byte store
                uint4* out = reinterpret_cast<uint4*>(img + e * kPix * 2);
                for (int i = threadIdx.x; i < kPix / 4; i += blockDim.x) {
                    const uint4 c = reinterpret_cast<const uint4*>(s_h)[i];
                    out[i] = make_uint4(enc(c.x & 0xFFFFu) | (enc(c.x >> 16) << 16),
                                        enc(c.y & 0xFFFFu) | (enc(c.y >> 16) << 16),
                                        enc(c.z & 0xFFFFu) | (enc(c.z >> 16) << 16),
                                        enc(c.w & 0xFFFFu) | (enc(c.w >> 16) << 16));
                }
            } else {
                uint16_t* out = img + e * kPix * 2;
                for (int i = threadIdx.x; i < kPix; i += blockDim.x) out[2 * i + pass] = (uint16_t)enc(s_h[i]);
            }
            __syncthreads();
        }
    }
}

void launch_bin_image(const float* hits, const int32_t* plane_off, int P, int D, const float* plane_z,
                      int64_t E, uint16_t* img, const uint32_t* err, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>(E, 2048);
    hipLaunchKernelGGL(k_bin_image, dim3(grid), dim3(256), 0, st, hits, plane_off, P, D, plane_z, E, img, err);
}

// Target heatmap: 1 at the bin of every target slope pair, else 0.
__global__ void k_target_image(const double* __restrict__ tg, const int64_t* __restrict__ off, int64_t E,
                               uint8_t* __restrict__ out)
{
    const double w = ((double)kSlopeHi - (double)kSlopeLo) / kImg;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        uint8_t* o = out + e * kPix;
        for (int i = threadIdx.x; i < kPix; i += blockDim.x) o[i] = 0;
        __syncthreads();
        for (int64_t t = off[e] + threadIdx.x; t < off[e + 1]; t += blockDim.x) {
            const double u = (tg[2 * t] - kSlopeLo) / w, v = (tg[2 * t + 1] - kSlopeLo) / w;
            if (u >= 0.0 && u < kImg && v >= 0.0 && v < kImg) o[(int)u * kImg + (int)v] = 1;
        }
        __syncthreads();
    }
}

void launch_target_image(const double* targets, const int64_t* off, int64_t E, uint8_t* tgt, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>(E, 2048);
    hipLaunchKernelGGL(k_target_image, dim3(grid), dim3(256), 0, st, targets, off, E, tgt);
}

// ------------------------------------------------------------ implicit GEMM
// C[m][n] = sum_k A(m, k) B(k, n) on 64 x 64 tiles, K tile 32, four waves of
// 32 x 32 (2 x 2 MFMA 16x16x16 bf16 blocks).  Both operands are staged in LDS
// with k contiguous (A as [m][k], B as [n][k]); an MFMA fragment is then one
// 8-byte LDS read per lane.  Index maps (pixel m = (b, r, c)):
//   kFwd     A(m, k) = x[b, r + dr, c + dc, ci]      k = tap * Cin + ci
//            B(k, n) = W[n][k]                         n = co
//   kBwdData A(m, k) = dz[b, r - dr, c - dc, co]     k = tap * Cout + co
//            B(k, n) = Wt[n][k] = W[co][tap * Cin + n] n = ci
//   kBwdW    A(m, k) = dz[p, m]                        m = co, k = pixel p of the chunk
//            B(k, n) = x[p + (dr, dc), ci]            n = tap * Cin + ci
// (zero outside the image and beyond the logical K).
constexpr int GBM = 64, GBN = 64, GBK = 32, GLD = GBK + 8;

struct GemmShape {
    int64_t M;
    int N, K;
};

__device__ __forceinline__ uint16_t load_px(const uint16_t* __restrict__ t, int64_t m, int dr, int dc, int ch,
                                            int C)
{
    const int64_t b = m / kPix;
    const int r = (int)((m / kImg) % kImg) + dr, c = (int)(m % kImg) + dc;
    if (r < 0 || r >= kImg || c < 0 || c >= kImg) return 0;
    return t[((b * kPix) + (int64_t)r * kImg + c) * C + ch];
}

// 8 consecutive channels [ch, ch + 8) of one (shifted) pixel: one 16-byte load
__device__ __forceinline__ uint4 load_px8(const uint16_t* __restrict__ t, int64_t m, int dr, int dc, int ch, int C)
{
    const int64_t b = m / kPix;
    const int r = (int)((m / kImg) % kImg) + dr, c = (int)(m % kImg) + dc;
    if (r < 0 || r >= kImg || c < 0 || c >= kImg) return make_uint4(0, 0, 0, 0);
    return *reinterpret_cast<const uint4*>(t + ((b * kPix) + (int64_t)r * kImg + c) * C + ch);
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs a, GemmShape s)
{
    __shared__ __align__(16) uint16_t As[GBM][GLD];
    __shared__ __align__(16) uint16_t Bs[GBN][GLD];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.x * GBM;
    const int n0 = blockIdx.y * GBN;
    const int chunk = blockIdx.z;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};

    const int cin = a.cin, cout = a.cout;
    for (int k0 = 0; k0 < s.K; k0 += GBK) {
        // ---- stage A and B (8 elements per thread each)
        if (a.mode == kFwd || a.mode == kBwdData) {
            // A: row = t / 4, k = k0 + (t % 4) * 8 .. + 7
            const int row = t >> 2, kk = k0 + (t & 3) * 8;
            const int64_t m = m0 + row;
            const int C = a.mode == kFwd ? cin : cout;
            const uint16_t* src = a.mode == kFwd ? a.x : a.dz;
            const int sgn = a.mode == kFwd ? 1 : -1;
            const int Klog = 9 * C;
            uint16_t v[8];
            if (C % 8 == 0 && kk + 8 <= Klog && m < s.M) {
                const int tap = kk / C, ch = kk % C;
                const uint4 q = load_px8(src, m, sgn * (tap / 3 - 1), sgn * (tap % 3 - 1), ch, C);
                *reinterpret_cast<uint4*>(v) = q;
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = kk + j;
                    v[j] = 0;
                    if (k < Klog && m < s.M) {
                        const int tap = k / C, ch = k % C;
                        v[j] = load_px(src, m, sgn * (tap / 3 - 1), sgn * (tap % 3 - 1), ch, C);
                    }
                }
            }
            *reinterpret_cast<uint4*>(&As[row][(t & 3) * 8]) = *reinterpret_cast<uint4*>(v);
            // B: row n = t / 4 of W (kFwd) or Wt (kBwdData), padded rows of length K
            const int n = n0 + row;
            uint4 q = make_uint4(0, 0, 0, 0);
            if (n < s.N) q = *reinterpret_cast<const uint4*>(a.w + (int64_t)n * s.K + kk);
            *reinterpret_cast<uint4*>(&Bs[row][(t & 3) * 8]) = q;
        } else {
            // kBwdW: thread -> pixel kk = k0 + t / 8, 8 consecutive rows (co) / columns (n)
            const int kkl = t >> 3, seg = (t & 7) * 8;
            const int64_t p = (int64_t)chunk * a.pix_per_chunk + k0 + kkl;
            // A rows m = co (dz[p][co .. co+7])
            uint16_t v[8];
            const int co0 = (int)m0 + seg;
            if (cout % 8 == 0 && co0 + 8 <= cout) {
                *reinterpret_cast<uint4*>(v) = *reinterpret_cast<const uint4*>(a.dz + p * cout + co0);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = co0 + j < cout ? a.dz[p * cout + co0 + j] : (uint16_t)0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) As[seg + j][kkl] = v[j];
            // B rows n = tap * cin + ci (x[p + shift][ci .. ci+7])
            const int nb = n0 + seg;
            const int Klog = 9 * cin;
            if (cin % 8 == 0 && nb + 8 <= Klog) {
                const int tap = nb / cin, ci = nb % cin;
                *reinterpret_cast<uint4*>(v) = load_px8(a.x, p, tap / 3 - 1, tap % 3 - 1, ci, cin);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int n = nb + j;
                    v[j] = 0;
                    if (n < Klog) {
                        const int tap = n / cin, ci = n % cin;
                        v[j] = load_px(a.x, p, tap / 3 - 1, tap % 3 - 1, ci, cin);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) Bs[seg + j][kkl] = v[j];
        }
        __syncthreads();
        // ---- 2 x 2 blocks x 2 K halves of MFMA 16x16x16
#pragma unroll
        for (int kh = 0; kh < 2; ++kh) {
            const int kq = kh * 16 + 4 * (lane >> 4);
            v4s af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                af[i] = *reinterpret_cast<const v4s*>(&As[wm * 32 + i * 16 + (lane & 15)][kq]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bf[j] = *reinterpret_cast<const v4s*>(&Bs[wn * 32 + j * 16 + (lane & 15)][kq]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // ---- epilogue: lane holds rows 4 * (lane / 16) + r, column lane % 16 of each block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wn * 32 + j * 16 + (lane & 15);
                if (m >= s.M || n >= s.N) continue;
                const float v = acc[i][j][r];
                if (a.mode == kFwd) {
                    const float z = v + a.bias[n];
                    if (a.act) a.y_bf16[m * cout + n] = f2bf(fmaxf(z, 0.0f));
                    else a.y_f32[m * cout + n] = z;
                } else if (a.mode == kBwdData) {
                    float g = v;
                    if (a.xprev && bf2f(a.xprev[m * cin + n]) <= 0.0f) g = 0.0f;
                    a.y_bf16[m * cin + n] = f2bf(g);
                } else {
                    a.partial[((int64_t)chunk * cout + m) * s.N + n] = v;
                }
            }
}

void launch_gemm(const GemmArgs& a, hipStream_t st)
{
    GemmShape s;
    dim3 grid;
    if (a.mode == kFwd) {
        s.M = (int64_t)a.B * kPix;
        s.N = a.cout;
        s.K = conv_kp(a.cin);
        grid = dim3((unsigned)(s.M / GBM), (unsigned)((s.N + GBN - 1) / GBN), 1);
    } else if (a.mode == kBwdData) {
        s.M = (int64_t)a.B * kPix;
        s.N = a.cin;
        s.K = conv_kp(a.cout);
        grid = dim3((unsigned)(s.M / GBM), (unsigned)((s.N + GBN - 1) / GBN), 1);
    } else {
        s.M = a.cout;
        s.N = conv_kp(a.cin);
        s.K = a.pix_per_chunk;
        const int64_t chunks = (int64_t)a.B * kPix / a.pix_per_chunk;
        grid = dim3((unsigned)((s.M + GBM - 1) / GBM), (unsigned)((s.N + GBN - 1) / GBN), (unsigned)chunks);
    }
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, a, s);
}

// ------------------------------------------------------- forward (inference)
// Direct convolutions for the forward pass, one kernel shape per layer kind:
//   k_conv_in   2 -> 64 channels: K = 18 is too short for MFMA; one thread per
//               (pixel, 8 output channels), FP32 FMAs, weights in LDS.
//   k_conv_mid  64 -> 128 and 128 -> 96: BF16 MFMA 32x32x16 (gfx950).  A
//               work-group (8 waves) owns 4 output rows x 128 columns x all
//               output channels.  The input rows it needs (with the zero halo)
//               sit in LDS once per 64-channel chunk and serve all nine taps;
//               the weights stream through LDS one (tap, chunk) slice at a
//               time, double-buffered.  Each wave computes 64 pixels x COUT;
//               the result goes back through LDS for coalesced 16-byte stores.
//   k_conv_head 96 -> 1: per pixel q the nine dot products U[q][tap] = sum_c
//               W[tap][c] x[q][c] (one read of the activations), then
//               logit[p] = b + sum_tap U[p + offset(tap)][tap] from LDS.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void k_conv_in(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
                                                 const float* __restrict__ bias, uint16_t* __restrict__ y,
                                                 int64_t npix)
{
    constexpr int CO = 64, K = 18, KP = conv_kp(2);
    __shared__ float s_w[CO * K];
    __shared__ float s_b[CO];
    for (int i = threadIdx.x; i < CO * K; i += blockDim.x) s_w[i] = bf2f(w[(i / K) * KP + i % K]);
    for (int i = threadIdx.x; i < CO; i += blockDim.x) s_b[i] = bias[i];
    __syncthreads();
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < npix * 8;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = g >> 3;
        const int cg = (int)(g & 7);
        const int64_t b = m / kPix;
        const int r = (int)((m / kImg) % kImg), c = (int)(m % kImg);
        float in[K];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int rr = r + tap / 3 - 1, cc = c + tap % 3 - 1;
            uint32_t v = 0;
            if (rr >= 0 && rr < kImg && cc >= 0 && cc < kImg)
                v = *reinterpret_cast<const uint32_t*>(x + ((b * kPix) + (int64_t)rr * kImg + cc) * 2);
            in[2 * tap] = bf2f((uint16_t)(v & 0xFFFFu));
            in[2 * tap + 1] = bf2f((uint16_t)(v >> 16));
        }
        uint16_t o[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float* wr = s_w + (8 * cg + j) * K;
            float acc = s_b[8 * cg + j];
#pragma unroll
            for (int k = 0; k < K; ++k) acc = fmaf(wr[k], in[k], acc);
            o[j] = f2bf(fmaxf(acc, 0.0f));
        }
        *reinterpret_cast<uint4*>(y + m * CO + 8 * cg) = *reinterpret_cast<const uint4*>(o);
    }
}

constexpr int kCvRows = 4;                 // output rows per work-group
constexpr int kCvThreads = 512;            // 8 waves: (output row, half row)
constexpr int kCvChunk = 64;               // input channels staged per pass
constexpr int kCvPitch = kCvChunk + 8;     // LDS elements per staged pixel (144 B)
constexpr int kCvCols = kImg + 2;          // staged columns incl. the zero halo

template <int CIN, int COUT>
constexpr size_t conv_mid_lds()
{
    constexpr size_t in = (size_t)(kCvRows + 2) * kCvCols * kCvPitch * 2;
    constexpr size_t wt = (size_t)2 * COUT * kCvPitch * 2;
    constexpr size_t out = (size_t)(kCvThreads / 64) * 64 * (COUT + 8) * 2;
    return in + wt > out ? in + wt : out;
}

template <int CIN, int COUT>
__global__ __launch_bounds__(kCvThreads) void k_conv_mid(const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ w,
                                                         const float* __restrict__ bias,
                                                         uint16_t* __restrict__ y)
{
    static_assert(CIN % kCvChunk == 0 && COUT % 32 == 0 && conv_kp(CIN) == 9 * CIN, "layer shape");
    constexpr int NB = COUT / 32, NCH = CIN / kCvChunk, KP = 9 * CIN;
    constexpr int WU = COUT * (kCvChunk / 8);                    // 16-byte units of one weight slice
    constexpr int WPT = (WU + kCvThreads - 1) / kCvThreads;
    constexpr int IU = (kCvRows + 2) * kCvCols * (kCvChunk / 8);  // 16-byte units of one input tile
    extern __shared__ float4 s_dyn[];
    uint16_t* s_in = reinterpret_cast<uint16_t*>(s_dyn);
    uint16_t* s_w = s_in + (kCvRows + 2) * kCvCols * kCvPitch;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int orow = wave >> 1, ocol0 = (wave & 1) * 64;
    const int64_t e = blockIdx.x / (kImg / kCvRows);
    const int r0 = (int)(blockIdx.x % (kImg / kCvRows)) * kCvRows;

    v16f acc[2][NB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    u32x4 wreg[WPT];
    for (int c = 0; c < NCH; ++c) {
        __syncthreads();
        for (int u = t; u < IU; u += kCvThreads) {
            const int q = u & 7, pc = (u >> 3) % kCvCols, pr = (u >> 3) / kCvCols;
            const int r = r0 - 1 + pr, col = pc - 1;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (r >= 0 && r < kImg && col >= 0 && col < kImg)
                v = *reinterpret_cast<const uint4*>(x + ((e * kImg + r) * kImg + col) * CIN + c * kCvChunk + q * 8);
            *reinterpret_cast<uint4*>(s_in + (pr * kCvCols + pc) * kCvPitch + q * 8) = v;
        }
        for (int tap = -1; tap < 9; ++tap) {
            // stage the next weight slice (tap + 1) while this tap computes
            if (tap < 8) {
#pragma unroll
                for (int i = 0; i < WPT; ++i) {
                    const int u = t + i * kCvThreads;
                    if (u < WU)
                        wreg[i] = *reinterpret_cast<const u32x4*>(w + (int64_t)(u >> 3) * KP + (tap + 1) * CIN +
                                                                  c * kCvChunk + (u & 7) * 8);
                }
            }
            if (tap >= 0) {
                const int dr = tap / 3 - 1, dc = tap % 3 - 1;
                const uint16_t* arow = s_in + ((orow + 1 + dr) * kCvCols + (ocol0 + 1 + dc)) * kCvPitch;
                const uint16_t* wb = s_w + (tap & 1) * COUT * kCvPitch;
#pragma unroll
                for (int kk = 0; kk < kCvChunk / 16; ++kk) {
                    const int ko = kk * 16 + 8 * (lane >> 5);
                    v8bf af[2], bfr[NB];
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb)
                        af[mb] = *reinterpret_cast<const v8bf*>(arow + (mb * 32 + (lane & 31)) * kCvPitch + ko);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        bfr[nb] = *reinterpret_cast<const v8bf*>(wb + (nb * 32 + (lane & 31)) * kCvPitch + ko);
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[mb], bfr[nb], acc[mb][nb], 0, 0, 0);
                }
            }
            if (tap < 8) {
                // buffer (tap + 1) & 1 was last read at tap - 1, before the barrier below it
                uint16_t* wn = s_w + ((tap + 1) & 1) * COUT * kCvPitch;
#pragma unroll
                for (int i = 0; i < WPT; ++i) {
                    const int u = t + i * kCvThreads;
                    if (u < WU) *reinterpret_cast<u32x4*>(wn + (u >> 3) * kCvPitch + (u & 7) * 8) = wreg[i];
                }
            }
            __syncthreads();
        }
    }
    // epilogue: bias, ReLU, BF16 through LDS; lane holds rows 8 (r / 4) + 4 (lane / 32) + r % 4,
    // column lane % 32 of each 32 x 32 block
    uint16_t* s_out = reinterpret_cast<uint16_t*>(s_dyn) + wave * 64 * (COUT + 8);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 32 + (lane & 31);
        const float bb = bias[co];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int px = mb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                s_out[px * (COUT + 8) + co] = f2bf(fmaxf(acc[mb][nb][r] + bb, 0.0f));
            }
    }
    __syncthreads();
    uint16_t* dst = y + ((e * kImg + r0 + orow) * kImg + ocol0) * COUT;
    constexpr int OU = 64 * COUT / 8;
    for (int u = lane; u < OU; u += 64) {
        const int px = u / (COUT / 8), q = u % (COUT / 8);
        *reinterpret_cast<uint4*>(dst + px * COUT + q * 8) =
            *reinterpret_cast<const uint4*>(s_out + px * (COUT + 8) + q * 8);
    }
}

constexpr int kHeadRows = 8;  // output rows per work-group of k_conv_head

__global__ __launch_bounds__(256) void k_conv_head(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
                                                   const float* __restrict__ bias, float* __restrict__ logits)
{
    constexpr int CIN = 96, KP = conv_kp(CIN), UR = kHeadRows + 2;
    __shared__ float s_w[9 * CIN];          // W[tap][c]
    __shared__ float s_u[UR * kImg * 9];    // U for the rows r0 - 1 .. r0 + kHeadRows
    const int64_t e = blockIdx.x / (kImg / kHeadRows);
    const int r0 = (int)(blockIdx.x % (kImg / kHeadRows)) * kHeadRows;
    for (int i = threadIdx.x; i < 9 * CIN; i += blockDim.x) s_w[i] = bf2f(w[i]);
    __syncthreads();
    for (int q = threadIdx.x; q < UR * kImg; q += blockDim.x) {
        const int r = r0 - 1 + q / kImg, col = q % kImg;
        float u[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) u[tap] = 0.0f;
        if (r >= 0 && r < kImg) {
            const uint16_t* px = x + ((e * kImg + r) * kImg + col) * CIN;
            for (int c8 = 0; c8 < CIN / 8; ++c8) {
                const uint4 raw = *reinterpret_cast<const uint4*>(px + c8 * 8);
                const uint16_t* h = reinterpret_cast<const uint16_t*>(&raw);
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = bf2f(h[j]);
#pragma unroll
                for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                    for (int j = 0; j < 8; ++j) u[tap] = fmaf(s_w[tap * CIN + c8 * 8 + j], v[j], u[tap]);
            }
        }
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) s_u[q * 9 + tap] = u[tap];
    }
    __syncthreads();
    const float b = bias[0];
    for (int p = threadIdx.x; p < kHeadRows * kImg; p += blockDim.x) {
        const int rl = p / kImg, col = p % kImg;  // output row r0 + rl = staged row rl + 1
        float z = b;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int sr = rl + 1 + tap / 3 - 1, cc = col + tap % 3 - 1;
            if (cc >= 0 && cc < kImg) z += s_u[(sr * kImg + cc) * 9 + tap];
        }
        logits[(e * kImg + r0 + rl) * kImg + col] = z;
    }
    static_assert(KP == 9 * CIN, "head weights are unpadded");
}

// ------------------------------------------------- fused inference kernels
// Inference needs only the logits, so two fusions keep activations on chip:
//   k_conv12  layer 1 computed into the LDS input tile of layer 2 (act1 never
//             reaches HBM); layer 1 runs on MFMA with K = 18 padded to 32;
//   k_conv3i  layer 3 (persistent, pipelined; below), whose epilogue
//             multiplies the BF16 act3 tile by the head's weights on MFMA
//             (U[q][tap], 9 floats per pixel) instead of storing act3, and
//             adds the nine shifted U values of every logit whose taps lie in
//             the band; k_head_edges finishes the band-edge rows.
// Training keeps every activation (k_conv_in, k_conv_mid<64, 128>, k_conv3,
// k_conv_head).
constexpr int kC12ImgRows = kCvRows + 4;          // image rows staged (halo 2)
constexpr int kC12ImgCols = kImg + 4;             // image columns staged
constexpr int kEdgeFloats = 13 * kImg;            // band-edge terms of the head per band (see k_conv3i)

constexpr int kC12Consts = 64 + 128 + 64 * 32 / 2;  // floats: b1, b2, then W1 (64 x 32 BF16)

constexpr size_t conv12_lds()
{
    return (size_t)(kCvRows + 2) * kCvCols * kCvPitch * 2 + (size_t)2 * 128 * kCvPitch * 2 +
           (size_t)kC12ImgRows * kC12ImgCols * 4 + (size_t)kC12Consts * 4;
}

__device__ __forceinline__ __bf16 bits_bf(uint16_t h) { return __builtin_bit_cast(__bf16, h); }

__device__ __forceinline__ uint2 pack4_bf16(float a, float b, float c, float d)
{
    return make_uint2((uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16), (uint32_t)f2bf(c) | ((uint32_t)f2bf(d) << 16));
}

// The fused kernels compute D = W x X^T (rows = output channels, columns =
// pixels), so a lane's 16 results are four runs of 4 consecutive channels of
// one pixel: channel 8 (r / 4) + 4 (lane / 32) + r % 4, pixel lane % 32.  Bias,
// ReLU and BF16 packing then give one 8-byte LDS store per run.
template <int NB, int COUT>
__device__ __forceinline__ void stage_act(uint16_t* s_out, const v16f (&acc)[NB][2], const float* __restrict__ bias,
                                          int lane)
{
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int co = nb * 32 + 8 * g + 4 * (lane >> 5);
            const float4 bb = *reinterpret_cast<const float4*>(bias + co);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int px = mb * 32 + (lane & 31);
                const v16f& a = acc[nb][mb];
                *reinterpret_cast<uint2*>(s_out + px * (COUT + 8) + co) =
                    pack4_bf16(fmaxf(a[4 * g] + bb.x, 0.0f), fmaxf(a[4 * g + 1] + bb.y, 0.0f),
                               fmaxf(a[4 * g + 2] + bb.z, 0.0f), fmaxf(a[4 * g + 3] + bb.w, 0.0f));
            }
        }
}

// layer 2's weight slice (tap) of all 128 output channels: 1024 16-byte units, two per thread
__device__ __forceinline__ void c12_load_w(const uint16_t* __restrict__ w2, int tap, int t, u32x4 (&r)[2])
{
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int u = t + i * kCvThreads;
        r[i] = *reinterpret_cast<const u32x4*>(w2 + (int64_t)(u >> 3) * 576 + tap * 64 + (u & 7) * 8);
    }
}

__device__ __forceinline__ void c12_store_w(uint16_t* dst, int t, const u32x4 (&r)[2])
{
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int u = t + i * kCvThreads;
        *reinterpret_cast<u32x4*>(dst + (u >> 3) * kCvPitch + (u & 7) * 8) = r[i];
    }
}

// act2 for inference is stored channel-chunked, [E][4][128][128][32], so that
// layer 3 reads whole runs per pixel and stage
__device__ __forceinline__ int64_t chunked_off(int64_t e, int chunk, int r, int col)
{
    return (((e * 4 + chunk) * kImg + r) * kImg + col) * 32;
}

// band processed by work-group `wg` in round `i` (G work-groups): the
// work-groups of XCD x (wg % 8 == x) take a contiguous run of bands
__device__ __forceinline__ int xcd_band(int wg, int i, int G)
{
    if (G % 8 != 0) return i * G + wg;
    const int per = G / 8;
    return i * G + (wg % 8) * per + wg / 8;
}

// Layers 1 and 2, persistent over 4-row bands, a run of consecutive bands per
// work-group.  Per band: layer 1 from the staged image rows into the LDS act1
// tile (the rows a band shares with the previous band of its event stay in
// the tile), then layer 2's nine taps, each
// tap's 128 x 64 weight slice double-buffered in LDS with the next slice
// (the next band's tap 0 after tap 8) loaded during this tap's products.
// The next band's image rows are loaded into registers while layer 2 runs and
// stored once the last tap has no use for the staging area; the results go
// from the accumulators straight to act2.
__global__ __launch_bounds__(kCvThreads) void k_conv12(const uint16_t* __restrict__ img,
                                                       const uint16_t* __restrict__ w1,
                                                       const float* __restrict__ b1,
                                                       const uint16_t* __restrict__ w2,
                                                       const float* __restrict__ b2, uint16_t* __restrict__ y,
                                                       int n_bands)
{
    constexpr int COUT = 128, NB = 4, BPE = kImg / kCvRows;
    constexpr int IMGU = kC12ImgRows * kC12ImgCols;              // staged image words (1056)
    constexpr int IPT = (IMGU + kCvThreads - 1) / kCvThreads;    // per thread (3)
    extern __shared__ float4 s_dyn[];
    uint16_t* s_in = reinterpret_cast<uint16_t*>(s_dyn);
    uint16_t* s_w = s_in + (kCvRows + 2) * kCvCols * kCvPitch;
    uint32_t* s_img = reinterpret_cast<uint32_t*>(s_w + 2 * COUT * kCvPitch);
    // biases and layer 1's weights in LDS for the whole kernel: read there, they
    // never make a wait on global memory (which would also wait for the act2
    // stores issued before them)
    float* s_b1 = reinterpret_cast<float*>(s_img + IMGU);
    float* s_b2 = s_b1 + 64;
    uint16_t* s_w1 = reinterpret_cast<uint16_t*>(s_b2 + COUT);
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int orow = wave >> 1, ocol0 = (wave & 1) * 64;
    const int G = gridDim.x;

    // image rows r0 - 2 .. r0 + 5, columns -2 .. 129 of a band (both channels in one word)
    uint32_t ireg[IPT];
    auto load_img = [&](int band) {
        const int64_t e = band / BPE;
        const int r0 = (band % BPE) * kCvRows;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int u = t + i * kCvThreads;
            const int r = r0 - 2 + u / kC12ImgCols, col = u % kC12ImgCols - 2;
            uint32_t v = 0;
            if (u < IMGU && r >= 0 && r < kImg && col >= 0 && col < kImg)
                v = *reinterpret_cast<const uint32_t*>(img + ((e * kImg + r) * kImg + col) * 2);
            ireg[i] = v;
        }
    };
    auto store_img = [&]() {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int u = t + i * kCvThreads;
            if (u < IMGU) s_img[u] = ireg[i];
        }
    };

    // consecutive bands per work-group: a band takes the two act1 rows it
    // shares with the previous band of its event from the tile
    const int b_hi = (int)((int64_t)(blockIdx.x + 1) * n_bands / G);
    int band = (int)((int64_t)blockIdx.x * n_bands / G);
    if (band >= b_hi) return;
    // the tile's halo columns (-1 and 128: layer 2's zero padding) are never written again
    if (t < (kCvRows + 2) * 2 * 8) {
        const int pos = t >> 3, chunk = t & 7;
        const int col = (pos & 1) ? kCvCols - 1 : 0;
        *reinterpret_cast<uint4*>(s_in + ((pos >> 1) * kCvCols + col) * kCvPitch + chunk * 8) = make_uint4(0u, 0u, 0u, 0u);
    }
    if (t < 64) s_b1[t] = b1[t];
    if (t < COUT) s_b2[t] = b2[t];
    if (t < 64 * 32 / 8) *reinterpret_cast<u32x4*>(s_w1 + 8 * t) = *reinterpret_cast<const u32x4*>(w1 + 8 * t);
    load_img(band);
    store_img();
    // weight slices in tap order, the same for every band: slice q of the
    // work-group's sequence sits in LDS buffer q & 1
    u32x4 wreg[2];
    c12_load_w(w2, 0, t, wreg);
    c12_store_w(s_w, t, wreg);
    c12_load_w(w2, 1, t, wreg);
    __syncthreads();

    int q = 0;     // weight slices consumed so far
    int base = 0;  // act1 row j of the band (image row r0 - 1 + j) sits in tile row (j + base) % 6
    for (int round = 0; band < b_hi; ++round) {
        const int64_t e = band / BPE;
        const int r0 = (band % BPE) * kCvRows;
        const int nband = band + 1;
        const bool more = nband < b_hi;
        // rows 4 and 5 of the previous band of the event are rows 0 and 1 of this one
        const bool fresh = round == 0 || band % BPE == 0;
        base = fresh ? 0 : (base + 4) % (kCvRows + 2);
        const int j0 = fresh ? 0 : 2;  // first act1 row computed here
        // the weight-slice reads and layer 1's image-read addresses below stay
        // inside the loop (the same every band, they would otherwise be hoisted
        // out of it and held in scratch memory across layer 2)
        int wz = 0;
        asm volatile("" : "+s"(wz));
        const uint16_t* w2r = w2 + wz;
        const uint32_t* s_imgr = s_img + wz;

        // layer 1 on the act1 tile (rows j0 .. 5 of image rows r0 - 1 .. r0 + 4,
        // columns 0 .. 127): D = W1 (64 x 32, K = 18 zero-padded) x X^T (32 x 32
        // positions) per block of 32 positions of one row; act1 outside the image
        // is the zero padding of layer 2
        v8bf aw[2][2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                aw[cb][ks] = *reinterpret_cast<const v8bf*>(s_w1 + (cb * 32 + (lane & 31)) * conv_kp(2) + ks * 16 +
                                                           8 * (lane >> 5));
        const int lz = lane + wz;  // = lane, recomputed each band (see above)
        constexpr int NW = kCvThreads / 64;
        constexpr int BPR = kImg / 32;  // position blocks per act1 row
        const int nblk = (kCvRows + 2 - j0) * BPR;  // 24 or 16: three or two per wave
        // block pb: its image reads, then its products and bias + ReLU + BF16
        // into the tile; a wave's first two blocks' reads are in flight together
        auto gather = [&](int pb, v8bf (&xv)[2]) {
            const int p = pb * 32 + (lz & 31);
            const int j = j0 + p / kImg, ic = p % kImg;  // act1 (r0 - 1 + j, ic)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const int tap = (ks * 16 + 8 * (lz >> 5)) / 2 + qq;
                    uint32_t v = 0;
                    // the tap adds (tap / 3 - 1, tap % 3 - 1); s_img starts at image (r0 - 2, -2)
                    if (tap < 9) v = s_imgr[(j + tap / 3) * kC12ImgCols + ic + 1 + tap % 3];
                    xv[ks][2 * qq] = bits_bf((uint16_t)(v & 0xFFFFu));
                    xv[ks][2 * qq + 1] = bits_bf((uint16_t)(v >> 16));
                }
        };
        auto finish = [&](int pb, const v8bf (&xv)[2]) {
            const int p = pb * 32 + (lz & 31);
            const int j = j0 + p / kImg, ic = p % kImg;
            const int ar = r0 - 1 + j;
            const bool inside = ar >= 0 && ar < kImg;
            int pr = j + base;
            if (pr >= kCvRows + 2) pr -= kCvRows + 2;
            uint16_t* dst = s_in + (pr * kCvCols + ic + 1) * kCvPitch;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                v16f a1;
#pragma unroll
                for (int r = 0; r < 16; ++r) a1[r] = 0.0f;
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw[cb][ks], xv[ks], a1, 0, 0, 0);
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int co = cb * 32 + 8 * g + 4 * (lz >> 5);
                    const float4 bb = *reinterpret_cast<const float4*>(s_b1 + co);
                    const uint2 v = inside ? pack4_bf16(fmaxf(a1[4 * g] + bb.x, 0.0f), fmaxf(a1[4 * g + 1] + bb.y, 0.0f),
                                                        fmaxf(a1[4 * g + 2] + bb.z, 0.0f),
                                                        fmaxf(a1[4 * g + 3] + bb.w, 0.0f))
                                           : make_uint2(0u, 0u);
                    *reinterpret_cast<uint2*>(dst + co) = v;
                }
            }
        };
        {
            v8bf xa[2], xb[2];
            gather(wave, xa);
            gather(wave + NW, xb);
            finish(wave, xa);
            finish(wave + NW, xb);
        }
        if (nblk > 2 * NW) {
            v8bf xc[2];
            gather(wave + 2 * NW, xc);
            finish(wave + 2 * NW, xc);
        }
        if (more) load_img(nband);  // in flight during layer 2
        __syncthreads();            // the act1 tile is complete

        // layer 2 (64 -> 128) on the act1 tile
        v16f acc[NB][2];
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
        for (int tap = 0; tap < 9; ++tap, ++q) {
            const int dr = tap / 3 - 1, dc = tap % 3 - 1;
            int lr = orow + 1 + dr + base;  // tile row of act1 row orow + 1 + dr
            if (lr >= kCvRows + 2) lr -= kCvRows + 2;
            const uint16_t* xrow = s_in + (lr * kCvCols + (ocol0 + 1 + dc)) * kCvPitch;
            const uint16_t* wb = s_w + (q & 1) * COUT * kCvPitch;
            // fragments of k-step kk + 1 are read while the products of kk run: the
            // scheduling barriers keep each read above the products it runs under
            v8bf xf[2][2], wf[2][NB];
            auto frags = [&](int kk, int set) __attribute__((always_inline)) {
                const int ko = kk * 16 + 8 * (lane >> 5);
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    xf[set][mb] = *reinterpret_cast<const v8bf*>(xrow + (mb * 32 + (lane & 31)) * kCvPitch + ko);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    wf[set][nb] = *reinterpret_cast<const v8bf*>(wb + (nb * 32 + (lane & 31)) * kCvPitch + ko);
            };
            frags(0, 0);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                if (kk < 3) frags(kk + 1, (kk + 1) & 1);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb)
                        acc[nb][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[kk & 1][nb], xf[kk & 1][mb],
                                                                             acc[nb][mb], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            // slice q + 1 into the buffer read during slice q - 1 (behind the
            // last barrier), then slice q + 2 requested
            if (tap < 8 || more) {
                c12_store_w(s_w + ((q + 1) & 1) * COUT * kCvPitch, t, wreg);
                if (tap < 7 || more) c12_load_w(w2r, (tap + 2) % 9, t, wreg);
            }
            if (tap == 8 && more) store_img();  // the image rows were last read by layer 1
            __syncthreads();
        }

        // epilogue: act2 = BF16(ReLU(acc + b2)).  In each 32-channel chunk a lane
        // holds channels 8 g + 4 h .. + 3 (g = 0..3, h = lane / 32) of its pixel;
        // the half-waves swap two of the four (lane ^ 32), so that each lane
        // writes two runs of eight channels, 16 j + 8 h .. + 7 (j = 0, 1), as
        // 16-byte stores
        const int h = lane >> 5;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            uint2 pk[2][4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float4 bb = *reinterpret_cast<const float4*>(s_b2 + nb * 32 + 8 * g + 4 * h);
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    const v16f& a = acc[nb][mb];
                    pk[mb][g] = pack4_bf16(fmaxf(a[4 * g] + bb.x, 0.0f), fmaxf(a[4 * g + 1] + bb.y, 0.0f),
                                           fmaxf(a[4 * g + 2] + bb.z, 0.0f), fmaxf(a[4 * g + 3] + bb.w, 0.0f));
                }
            }
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                // h = 0 keeps g = 0, 2 and sends g = 1, 3; h = 1 the other way round
                const uint2 s0 = h ? pk[mb][0] : pk[mb][1];
                const uint2 s1 = h ? pk[mb][2] : pk[mb][3];
                const uint2 q0 = make_uint2((uint32_t)__shfl_xor((int)s0.x, 32), (uint32_t)__shfl_xor((int)s0.y, 32));
                const uint2 q1 = make_uint2((uint32_t)__shfl_xor((int)s1.x, 32), (uint32_t)__shfl_xor((int)s1.y, 32));
                const uint4 run0 = h ? make_uint4(q0.x, q0.y, pk[mb][1].x, pk[mb][1].y)
                                     : make_uint4(pk[mb][0].x, pk[mb][0].y, q0.x, q0.y);
                const uint4 run1 = h ? make_uint4(q1.x, q1.y, pk[mb][3].x, pk[mb][3].y)
                                     : make_uint4(pk[mb][2].x, pk[mb][2].y, q1.x, q1.y);
                uint16_t* dst = y + chunked_off(e, nb, r0 + orow, ocol0 + mb * 32 + (lane & 31)) + 8 * h;
                *reinterpret_cast<uint4*>(dst) = run0;
                *reinterpret_cast<uint4*>(dst + 16) = run1;
            }
        }
        band = nband;
    }
}

constexpr int kC3Chunk = 32;                    // input channels per chunk
constexpr int kC3Pitch = kC3Chunk + 8;          // LDS elements per staged pixel (80 B)
constexpr int kC3Tile = (kCvRows + 2) * kCvCols * kC3Pitch;   // elements of one staged chunk
constexpr int kC3TU = (kCvRows + 2) * kCvCols * (kC3Chunk / 8);  // 16-byte units of one chunk (3120)
constexpr int kC3TPT = (kC3TU + kCvThreads - 1) / kCvThreads;    // per thread (7)

constexpr size_t conv3_lds()
{
    constexpr size_t main = (size_t)2 * kC3Tile * 2 + (size_t)2 * 96 * kC3Pitch * 2;
    constexpr size_t out = (size_t)(kCvThreads / 64) * 64 * (96 + 8) * 2;
    return main > out ? main : out;
}

// Layer 3 for training: act2 NHWC in, act3 NHWC out (inference runs k_conv3i).
__global__ __launch_bounds__(kCvThreads) void k_conv3(const uint16_t* __restrict__ x,
                                                      const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias,
                                                      uint16_t* __restrict__ y)
{
    constexpr int CIN = 128, COUT = 96, NB = 3, NCH = CIN / kC3Chunk, KP = 9 * CIN;
    constexpr int WU = COUT * (kC3Chunk / 8);  // 384 units per weight slice
    extern __shared__ float4 s_dyn[];
    uint16_t* s_in = reinterpret_cast<uint16_t*>(s_dyn);
    uint16_t* s_w = s_in + 2 * kC3Tile;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int orow = wave >> 1, ocol0 = (wave & 1) * 64;
    const int64_t e = blockIdx.x / (kImg / kCvRows);
    const int r0 = (int)(blockIdx.x % (kImg / kCvRows)) * kCvRows;

    uint4 treg[kC3TPT];
    auto load_tile = [&](int c) {
#pragma unroll
        for (int i = 0; i < kC3TPT; ++i) {
            const int u = t + i * kCvThreads;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (u < kC3TU) {
                const int q = u & 3, pc = (u >> 2) % kCvCols, pr = (u >> 2) / kCvCols;
                const int r = r0 - 1 + pr, col = pc - 1;
                if (r >= 0 && r < kImg && col >= 0 && col < kImg) {
                    const int64_t off = ((e * kImg + r) * kImg + col) * CIN + c * kC3Chunk + q * 8;
                    v = *reinterpret_cast<const uint4*>(x + off);
                }
            }
            treg[i] = v;
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int i = 0; i < kC3TPT; ++i) {
            const int u = t + i * kCvThreads;
            if (u < kC3TU) {
                const int q = u & 3, pix = u >> 2;
                *reinterpret_cast<uint4*>(s_in + buf * kC3Tile + pix * kC3Pitch + q * 8) = treg[i];
            }
        }
    };
    uint4 wreg[9];
    auto store_w = [&](int buf, const uint4& v) {
        if (t < WU) *reinterpret_cast<uint4*>(s_w + buf * COUT * kC3Pitch + (t >> 2) * kC3Pitch + (t & 3) * 8) = v;
    };

    v16f acc[NB][2];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    load_tile(0);
    store_tile(0);
    for (int c = 0; c < NCH; ++c) {
        // this chunk's nine weight slices first, then the next chunk's rows: the
        // per-tap waits for the weights then never wait for the row loads
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            wreg[tap] = t < WU ? *reinterpret_cast<const uint4*>(w + (int64_t)(t >> 2) * KP + tap * CIN +
                                                                 c * kC3Chunk + (t & 3) * 8)
                               : make_uint4(0, 0, 0, 0);
        if (c + 1 < NCH) load_tile(c + 1);
        store_w(0, wreg[0]);
        __syncthreads();
        const uint16_t* tile = s_in + (c & 1) * kC3Tile;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dr = tap / 3 - 1, dc = tap % 3 - 1;
            const uint16_t* xrow = tile + ((orow + 1 + dr) * kCvCols + (ocol0 + 1 + dc)) * kC3Pitch;
            const uint16_t* wb = s_w + (tap & 1) * COUT * kC3Pitch;
#pragma unroll
            for (int kk = 0; kk < kC3Chunk / 16; ++kk) {
                const int ko = kk * 16 + 8 * (lane >> 5);
                v8bf xf[2], wf[NB];
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    xf[mb] = *reinterpret_cast<const v8bf*>(xrow + (mb * 32 + (lane & 31)) * kC3Pitch + ko);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    wf[nb] = *reinterpret_cast<const v8bf*>(wb + (nb * 32 + (lane & 31)) * kC3Pitch + ko);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb)
                        acc[nb][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[nb], xf[mb], acc[nb][mb], 0, 0, 0);
            }
            if (tap < 8) store_w((tap + 1) & 1, wreg[tap + 1]);
            __syncthreads();
        }
        // the other tile buffer was last read in chunk c - 1, before the barriers above
        if (c + 1 < NCH) store_tile((c + 1) & 1);
    }

    uint16_t* s_out = reinterpret_cast<uint16_t*>(s_dyn) + wave * 64 * (COUT + 8);
    stage_act<NB, COUT>(s_out, acc, bias, lane);
    __syncthreads();
    const int64_t pix0 = (e * kImg + r0 + orow) * kImg + ocol0;
    uint16_t* dst = y + pix0 * COUT;
    for (int u = lane; u < 64 * COUT / 8; u += 64) {
        const int px = u / (COUT / 8), q = u % (COUT / 8);
        *reinterpret_cast<uint4*>(dst + px * COUT + q * 8) = *reinterpret_cast<const uint4*>(s_out + px * (COUT + 8) + q * 8);
    }
}

// ---------------------------------------------- layer 3, inference, pipelined
// Layer 3 (128 -> 96) and the head product U[q][tap] = sum_c W4[tap][c]
// act3[q][c] for bands of kCvRows output rows, persistent: work-group w takes
// bands w, w + G, w + 2G, ... of the batch, so a band's input halo rows come
// from the neighbouring bands that the other work-groups of its XCD process
// at the same time (work-groups are dealt to the XCDs round-robin, and the
// band order below gives each XCD a contiguous range of bands).  The 128
// input channels stream through LDS in stages of 16: the stage's input rows
// and all nine taps' weights (double-buffered, one barrier per stage), the
// next stage (or the next band's first stage) loaded from global memory while
// this one's products run, and each tap's fragments read from LDS one tap
// ahead of its products.  The epilogue takes the head product straight from
// the accumulators: a lane's 16 results are four runs of four channels of one
// pixel, so with the contraction index ordered the same way in W4's fragment,
// each 8-value half of a run pair is already a B fragment of the product.
constexpr int kL3Stage = 16;                                       // input channels per stage
constexpr int kL3Pitch = kL3Stage;  // LDS elements per pixel / weight row (32 B: a fragment read's 8 lanes hit distinct banks)
constexpr int kL3Rows = kCvRows + 2;                               // staged input rows (halo 1)
constexpr int kL3InUnits = kL3Rows * kCvCols * (kL3Stage / 8);     // 16-byte units of a stage's input (1560)
constexpr int kL3WUnits = 9 * 96 * (kL3Stage / 8);                 // ... of its weights (1728)
constexpr int kL3InPT = (kL3InUnits + kCvThreads - 1) / kCvThreads;
constexpr int kL3WPT = (kL3WUnits + kCvThreads - 1) / kCvThreads;
constexpr int kL3InElems = kL3Rows * kCvCols * kL3Pitch;           // one input buffer
constexpr int kL3WElems = 9 * 96 * kL3Pitch;                       // one weight buffer

constexpr int kL3HeadFrags = 6 * 64;                               // head-weight fragments (nb, ks, lane), 16 B each

constexpr int kL3UFloats = 9 * kCvRows * kImg;  // the band's U, tap-major
constexpr size_t conv3i_lds()
{
    return (size_t)2 * (kL3InElems + kL3WElems) * 2 + (size_t)kL3HeadFrags * 16 + 96 * 4 + (size_t)kL3UFloats * 4;
}

__global__ __launch_bounds__(kCvThreads) void k_conv3i(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       const uint16_t* __restrict__ w4,
                                                       const float* __restrict__ hbias, float* __restrict__ edge,
                                                       float* __restrict__ logits, int n_bands)
{
    constexpr int CIN = 128, COUT = 96, NB = 3, NST = CIN / kL3Stage, KP = 9 * CIN;
    constexpr int BPE = kImg / kCvRows;  // bands per event
    static_assert(NST % 2 == 0, "a band's first stage must land in buffer 0");
    extern __shared__ float4 s_dyn[];
    uint16_t* s_in = reinterpret_cast<uint16_t*>(s_dyn);
    uint16_t* s_w = s_in + 2 * kL3InElems;
    // the head's weight fragments and layer 3's bias, in LDS for the whole kernel
    v8bf* s_hf = reinterpret_cast<v8bf*>(s_w + 2 * kL3WElems);
    float* s_b3 = reinterpret_cast<float*>(s_hf + kL3HeadFrags);
    float* s_u = s_b3 + 96;  // U of the band's 4 x 128 pixels, [tap][row][column]
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int orow = wave >> 1, ocol0 = (wave & 1) * 64;
    const int G = gridDim.x;

    // a stage is moved in two halves (units i = 2 k, 2 k + 1 of each thread's
    // input and weight units), each through its own set of registers
    static_assert(kL3InPT == 4 && kL3WPT == 4, "two halves of two units each");
    u32x4 ra_in[2], ra_w[2], rb_in[2], rb_w[2];
    auto load_half = [&](int band, int c, int k, u32x4 (&pin)[2], u32x4 (&pw)[2]) {
        const int64_t e = band / BPE;
        const int r0 = (band % BPE) * kCvRows;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int u = t + (2 * k + i) * kCvThreads;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (u < kL3InUnits) {
                const int q = u & 1, pix = u >> 1;
                const int r = r0 - 1 + pix / kCvCols, col = pix % kCvCols - 1;
                if (r >= 0 && r < kImg && col >= 0 && col < kImg)
                    v = *reinterpret_cast<const u32x4*>(x + chunked_off(e, c >> 1, r, col) + (c & 1) * kL3Stage + q * 8);
            }
            pin[i] = v;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int u = t + (2 * k + i) * kCvThreads;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (u < kL3WUnits) {
                const int q = u & 1, row = u >> 1;  // row = tap * COUT + co
                const int tap = row / COUT, co = row % COUT;
                v = *reinterpret_cast<const u32x4*>(w + (int64_t)co * KP + tap * CIN + c * kL3Stage + q * 8);
            }
            pw[i] = v;
        }
    };
    auto store_half = [&](int buf, int k, const u32x4 (&pin)[2], const u32x4 (&pw)[2]) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int u = t + (2 * k + i) * kCvThreads;
            if (u < kL3InUnits)
                *reinterpret_cast<u32x4*>(s_in + buf * kL3InElems + (u >> 1) * kL3Pitch + (u & 1) * 8) = pin[i];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int u = t + (2 * k + i) * kCvThreads;
            if (u < kL3WUnits)
                *reinterpret_cast<u32x4*>(s_w + buf * kL3WElems + (u >> 1) * kL3Pitch + (u & 1) * 8) = pw[i];
        }
    };

    int band = xcd_band(blockIdx.x, 0, G);
    if (band >= n_bands) return;
    if (t < kL3HeadFrags) {
        // fragment (nb, ks) of lane l: k position 4 g + q is head weight (tap
        // l % 32, channel nb 32 + 8 (2 ks + g) + 4 (l / 32) + q), zero for taps >= 9
        const int nb = t / 128, ks = (t / 64) % 2, l = t % 64, n = l & 31, hh = l >> 5;
        v8bf f;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                f[4 * g + q] = n < 9 ? bits_bf(w4[n * COUT + nb * 32 + 8 * (2 * ks + g) + 4 * hh + q]) : bits_bf(0);
        s_hf[t] = f;
    }
    if (t < COUT) s_b3[t] = bias[t];
    const float b4 = hbias[0];
    load_half(band, 0, 0, ra_in, ra_w);
    store_half(0, 0, ra_in, ra_w);
    load_half(band, 0, 1, rb_in, rb_w);
    store_half(0, 1, rb_in, rb_w);
    load_half(band, 1, 0, ra_in, ra_w);  // stage 1 in flight
    load_half(band, 1, 1, rb_in, rb_w);
    __syncthreads();
    // logits of band pb whose nine taps lie in the band, added in tap order
    // (zero outside the image) from its U in LDS, and the first six terms of
    // its last row when a band lies below.  Run behind a barrier that follows
    // the band's epilogue: the first stage barrier of the next band, or the one
    // after the last band.
    auto head_logits = [&](int pb) {
        static_assert(kCvThreads == kCvRows * kImg, "one thread per pixel of the band");
        const int64_t pe = pb / BPE;
        const int kb = pb % BPE;
        const bool above = kb > 0, below = kb < BPE - 1;
        int wz = 0;
        asm volatile("" : "+s"(wz));
        const int tz = t + wz;  // see the epilogue
        const int row = tz / kImg, col = tz % kImg;
        const bool edge_row = (row == 0 && above) || (row == kCvRows - 1 && below);
        float z = b4;
        const int ntap = edge_row ? (row == 0 ? 0 : 6) : 9;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int rr = row + tap / 3 - 1, cc = col + tap % 3 - 1;
            if (tap < ntap && rr >= 0 && rr < kCvRows && cc >= 0 && cc < kImg)
                z += s_u[(tap * kCvRows + rr) * kImg + cc];
        }
        if (!edge_row) logits[(pe * kImg + kb * kCvRows + row) * kImg + col] = z;
        else if (row == kCvRows - 1) edge[(int64_t)pb * kEdgeFloats + 12 * kImg + col] = z;
    };
    int prev = -1;  // the band whose logits are still to be summed from U
    for (int round = 0; band < n_bands; band = xcd_band(blockIdx.x, ++round, G)) {
        v16f acc[NB][2];
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
        const int nxt = xcd_band(blockIdx.x, round + 1, G);
#pragma unroll
        for (int c = 0; c < NST; ++c) {
            // stage s + 1 (in registers since stage s - 1) goes into the buffer not
            // read in this stage, and stage s + 2 is requested: each half of a stage
            // has a whole stage of products to arrive.  Stages run on into the
            // next band's first ones.
            const int b1 = c + 1 < NST ? band : nxt;
            const int b2 = c + 2 < NST ? band : nxt, c2 = (c + 2) % NST;
            const bool m1 = b1 < n_bands, m2 = b2 < n_bands;
            if (m1) store_half((c + 1) & 1, 0, ra_in, ra_w);
            if (m2) load_half(b2, c2, 0, ra_in, ra_w);
            __builtin_amdgcn_sched_barrier(0);  // the loads go out first
            const uint16_t* ti = s_in + (c & 1) * kL3InElems;
            const uint16_t* tw = s_w + (c & 1) * kL3WElems;
            v8bf xf[2][2], wf[2][NB];
            auto frags = [&](int tap, int set) {
                const int dr = tap / 3 - 1, dc = tap % 3 - 1;
                const uint16_t* xrow = ti + ((orow + 1 + dr) * kCvCols + (ocol0 + 1 + dc)) * kL3Pitch + 8 * (lane >> 5);
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    xf[set][mb] = *reinterpret_cast<const v8bf*>(xrow + (mb * 32 + (lane & 31)) * kL3Pitch);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    wf[set][nb] = *reinterpret_cast<const v8bf*>(tw + (tap * COUT + nb * 32 + (lane & 31)) * kL3Pitch +
                                                                 8 * (lane >> 5));
            };
            frags(0, 0);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                if (tap == 4) {
                    if (m1) store_half((c + 1) & 1, 1, rb_in, rb_w);
                    if (m2) load_half(b2, c2, 1, rb_in, rb_w);
                }
                if (tap < 8) frags(tap + 1, (tap + 1) & 1);
                // keep the next tap's reads above this tap's products (the
                // scheduler would otherwise sink each read to its first use)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb)
                        acc[nb][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[tap & 1][nb], xf[tap & 1][mb],
                                                                             acc[nb][mb], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            // the buffer filled here was last read in the previous stage, before the barrier below it
            __syncthreads();
            if (c == 0 && prev >= 0) head_logits(prev);  // U of the previous band is complete
        }

        // epilogue: act3 = BF16(ReLU(acc + b3)), U^T (9 taps padded to 32 rows x
        // 32 pixels) = W4 x act3^T per pixel block; W4's fragments and b3 from LDS
        const int kb = band % BPE;
        const bool above = kb > 0, below = kb < BPE - 1;  // neighbour bands in the event
        float* eb = edge + (int64_t)band * kEdgeFloats;
        // lane-dependent addresses formed anew per band (an opaque zero: hoisted
        // out of the band loop they would be held in scratch memory)
        int wz = 0;
        asm volatile("" : "+s"(wz));
        const int lz = lane + wz;
        const int h = lz >> 5, n = lz & 31;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            v16f au;
#pragma unroll
            for (int r = 0; r < 16; ++r) au[r] = 0.0f;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    // k position j of this lane's half = result r = 8 ks + j: channel
                    // nb 32 + 8 (r / 4) + 4 h + r % 4 (the same order in W4's fragment)
                    v8bf xa;
                    const v8bf wa = s_hf[(nb * 2 + ks) * 64 + lane];
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        const int ch = nb * 32 + 8 * (2 * ks + g) + 4 * h;
                        const float4 bb = *reinterpret_cast<const float4*>(s_b3 + ch);
                        const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            xa[4 * g + q] = bits_bf(f2bf(fmaxf(acc[nb][mb][8 * ks + 4 * g + q] + bv[q], 0.0f)));
                    }
                    au = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, xa, au, 0, 0, 0);
                }
            }
            // lane < 32 holds taps 0-3 and 8 of pixel n, lane >= 32 taps 4-7
            const int col = ocol0 + mb * 32 + n;
            // band-edge terms (per band, 13 rows of 128 floats): 0-5 taps 3-8 of
            // row 0, 6-8 taps 6-8 of row 1 (when a band lies above: its last
            // logit row needs row 0's taps 6-8, and this band's first logit row
            // is finished after that band's taps 0-2), 9-11 taps 0-2 of row 3
            // (when a band lies below), 12 the partial sum of row 3
            auto put = [&](int tap, float v) {
                s_u[(tap * kCvRows + orow) * kImg + col] = v;
                if (orow == 0 && above && tap >= 3) eb[(tap - 3) * kImg + col] = v;
                if (orow == 1 && above && tap >= 6) eb[tap * kImg + col] = v;
                if (orow == 3 && below && tap < 3) eb[(9 + tap) * kImg + col] = v;
            };
#pragma unroll
            for (int q = 0; q < 4; ++q) put(4 * h + q, au[q]);
            if (h == 0) put(8, au[4]);
        }
        prev = band;
    }
    if (prev >= 0) {
        // the last band's U: an LDS-only barrier (the epilogue's stores need no wait)
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        head_logits(prev);
    }
}

// The head's band-edge logit rows, from the terms k_conv3i wrote per band:
// the first row of a band with a band above adds, after the bias, that band's
// row-3 taps 0-2 and then its own row-0 taps 3-5 and row-1 taps 6-8; the last
// row of a band with a band below continues its partial sum with that band's
// row-0 taps 6-8 (tap order, zero outside the image).
__global__ __launch_bounds__(256) void k_head_edges(const float* __restrict__ edge, const float* __restrict__ bias,
                                                    int64_t n_bands, float* __restrict__ logits)
{
    constexpr int BPE = kImg / kCvRows;
    const float b = bias[0];
    const int64_t n = n_bands * 2 * kImg;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t band = i / (2 * kImg);
        const int last = (int)((i / kImg) & 1), col = (int)(i % kImg);
        const int kb = (int)(band % BPE);
        const int64_t e = band / BPE;
        const float* eb = edge + band * kEdgeFloats;
        // every term is read first (at a clamped column), then added in tap
        // order where its column lies in the image: the reads go out together
        float z;
        if (!last) {
            if (kb == 0) continue;
            const float* ea = eb - kEdgeFloats;  // the band above
            float v[9];
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int cc = min(max(col + tap % 3 - 1, 0), kImg - 1);
                v[tap] = tap < 3 ? ea[(9 + tap) * kImg + cc] : eb[(tap < 6 ? tap - 3 : tap) * kImg + cc];
            }
            z = b;
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int cc = col + tap % 3 - 1;
                z = (cc >= 0 && cc < kImg) ? z + v[tap] : z;
            }
            logits[(e * kImg + kb * kCvRows) * kImg + col] = z;
        } else {
            if (kb == BPE - 1) continue;
            const float* en = eb + kEdgeFloats;  // the band below
            float v[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) v[k] = en[(3 + k) * kImg + min(max(col + k - 1, 0), kImg - 1)];
            z = eb[12 * kImg + col];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int cc = col + k - 1;
                z = (cc >= 0 && cc < kImg) ? z + v[k] : z;
            }
            logits[(e * kImg + kb * kCvRows + kCvRows - 1) * kImg + col] = z;
        }
    }
}

// One-time set-up of the forward kernels (dynamic LDS limits) and the CU
// count; idempotent, and called before any stream capture of the forward.
int prepare_forward()
{
    // a function-local static: initialised once, thread-safe
    static const int n_cu = [] {
        constexpr size_t l1 = conv_mid_lds<64, 128>(), l12 = conv12_lds(), l3 = conv3_lds(), l3i = conv3i_lds();
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
            n = 256;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_conv3i), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)l3i);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_conv_mid<64, 128>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)l1);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_conv12), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)l12);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_conv3), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)l3);
        (void)hipGetLastError();
        return n;
    }();
    return n_cu;
}

void launch_forward(const uint16_t* img, const uint16_t* wbf, const float* w32, const NetLayout& L, int64_t E,
                    uint16_t* act1, uint16_t* act2, uint16_t* act3, float* u, float* logits, bool train,
                    hipStream_t st)
{
    constexpr size_t l1 = conv_mid_lds<64, 128>(), l12 = conv12_lds(), l3 = conv3_lds(), l3i = conv3i_lds();
    const int n_cu = prepare_forward();
    const int64_t npix = E * kPix;
    const unsigned gm = (unsigned)(E * (kImg / kCvRows));
    if (train) {
        const int g0 = (int)std::min<int64_t>((npix * 8 + 255) / 256, 65536);
        hipLaunchKernelGGL(k_conv_in, dim3(g0), dim3(256), 0, st, img, wbf + L.w_off[0], w32 + L.b_off[0], act1, npix);
        hipLaunchKernelGGL((k_conv_mid<64, 128>), dim3(gm), dim3(kCvThreads), l1, st, act1, wbf + L.w_off[1],
                           w32 + L.b_off[1], act2);
        hipLaunchKernelGGL(k_conv3, dim3(gm), dim3(kCvThreads), l3, st, act2, wbf + L.w_off[2], w32 + L.b_off[2], act3);
        hipLaunchKernelGGL(k_conv_head, dim3((unsigned)(E * (kImg / kHeadRows))), dim3(256), 0, st, act3,
                           wbf + L.w_off[3], w32 + L.b_off[3], logits);
    } else {
        // both persistent, one work-group per CU (their LDS tiles fill it)
        const int n_bands = (int)gm;
        const unsigned g12 = (unsigned)std::min<int64_t>(n_bands, (int64_t)n_cu);
        hipLaunchKernelGGL(k_conv12, dim3(g12), dim3(kCvThreads), l12, st, img, wbf + L.w_off[0], w32 + L.b_off[0],
                           wbf + L.w_off[1], w32 + L.b_off[1], act2, n_bands);
        const unsigned g3 = (unsigned)std::min<int64_t>(n_bands, (int64_t)n_cu);
        hipLaunchKernelGGL(k_conv3i, dim3(g3), dim3(kCvThreads), l3i, st, act2, wbf + L.w_off[2], w32 + L.b_off[2],
                           wbf + L.w_off[3], w32 + L.b_off[3], u, logits, n_bands);
        const int gh = (int)std::min<int64_t>(((int64_t)n_bands * 2 * kImg + 255) / 256, 65536);
        hipLaunchKernelGGL(k_head_edges, dim3(gh), dim3(256), 0, st, u, w32 + L.b_off[3], (int64_t)n_bands, logits);
    }
}

// ------------------------------------------------------------------ losses
// Weighted binary cross-entropy on logits z with targets y in {0, 1}:
//   l = w y softplus(-z) + (1 - y) softplus(z),  dl/dz = (w y + 1 - y) sigma(z) - w y
// mean over all pixels; per-block partial sums of l (fixed order reduction).
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ z, const uint8_t* __restrict__ y,
                                             int64_t n, float pw, float* __restrict__ part,
                                             uint16_t* __restrict__ dz)
{
    __shared__ float s[256];
    float acc = 0.0f;
    const float inv = 1.0f / (float)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float zi = z[i];
        const float yi = (float)y[i];
        const float sp_pos = fmaxf(zi, 0.0f) + log1pf(expf(-fabsf(zi)));  // softplus(z)
        const float sp_neg = sp_pos - zi;                                  // softplus(-z)
        acc += pw * yi * sp_neg + (1.0f - yi) * sp_pos;
        const float sig = 1.0f / (1.0f + expf(-zi));
        dz[i] = f2bf(((pw * yi + 1.0f - yi) * sig - pw * yi) * inv);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0] * inv;
}

void launch_bce(const float* z, const uint8_t* y, int64_t n, float pw, float* part, uint16_t* dz, hipStream_t st)
{
    hipLaunchKernelGGL(k_bce, dim3(1024), dim3(256), 0, st, z, y, n, pw, part, dz);
}

__global__ void k_sum(const float* __restrict__ part, int n, float* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s;
    }
}

void launch_sum(const float* part, int n, float* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, st, part, n, out);
}

// Wt[ci][tap * Cout + co] = W[co][tap * Cin + ci] (rows padded to conv_kp(Cout))
__global__ void k_transpose_w(const uint16_t* __restrict__ w, int cin, int cout, uint16_t* __restrict__ wt)
{
    const int kpo = conv_kp(cout), kpi = conv_kp(cin);
    const int64_t n = (int64_t)cin * kpo;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i / kpo), k = (int)(i % kpo);
        uint16_t v = 0;
        if (k < 9 * cout) {
            const int tap = k / cout, co = k % cout;
            v = w[(int64_t)co * kpi + tap * cin + ci];
        }
        wt[i] = v;
    }
}

void launch_transpose_w(const uint16_t* w, int cin, int cout, uint16_t* wt, hipStream_t st)
{
    hipLaunchKernelGGL(k_transpose_w, dim3(256), dim3(256), 0, st, w, cin, cout, wt);
}

// grad[i] = sum over chunks c (in order) of partial[c][i]
__global__ void k_reduce_dw(const float* __restrict__ part, int nc, int64_t n, float* __restrict__ g)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int c = 0; c < nc; ++c) s += part[(int64_t)c * n + i];
        g[i] = s;
    }
}

void launch_reduce_dw(const float* part, int nc, int64_t n, float* g, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_dw, dim3(512), dim3(256), 0, st, part, nc, n, g);
}

// bias gradient: per chunk of pixels a partial sum of dz over the chunk (one
// thread per channel, pixels in order), then an ordered sum over chunks
// Bias gradient, per chunk of pixels: the chunk's dz values are one contiguous
// run of per x cout BF16 values; the block's threads walk it with a stride of
// (256 / cout) cout, so each thread stays on one channel (t % cout), with four
// running sums over alternate elements; then the threads of a channel are
// added in a fixed order in LDS.
__global__ __launch_bounds__(256) void k_bias_part(const uint16_t* __restrict__ dz, int64_t npix, int cout,
                                                   int nchunk, float* __restrict__ part)
{
    __shared__ float s_sum[256];
    const int t = threadIdx.x;
    const int c = blockIdx.x;
    const int groups = 256 / cout;  // threads per channel
    const int stride = groups * cout;
    const int64_t per = npix / nchunk;
    const int64_t n = per * cout;
    const uint16_t* src = dz + (int64_t)c * n;
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (t < stride) {
        int64_t i = t;
        for (; i + 3 * stride < n; i += 4 * stride) {
#pragma unroll
            for (int k = 0; k < 4; ++k) s[k] += bf2f(src[i + k * stride]);
        }
        if (i < n) s[0] += bf2f(src[i]);
        if (i + stride < n) s[1] += bf2f(src[i + stride]);
        if (i + 2 * stride < n) s[2] += bf2f(src[i + 2 * stride]);
    }
    s_sum[t] = (s[0] + s[1]) + (s[2] + s[3]);
    __syncthreads();
    if (t < cout) {
        float v = 0.0f;
        for (int g = 0; g < groups; ++g) v += s_sum[g * cout + t];
        part[(int64_t)c * cout + t] = v;
    }
}

__global__ void k_bias_reduce(const float* __restrict__ part, int cout, int nchunk, float* __restrict__ g)
{
    const int co = threadIdx.x;
    if (co >= cout) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * cout + co];
    g[co] = s;
}

void launch_bias_grad(const uint16_t* dz, int64_t npix, int cout, int nchunk, float* part, float* gb, hipStream_t st)
{
    hipLaunchKernelGGL(k_bias_part, dim3(nchunk), dim3(256), 0, st, dz, npix, cout, nchunk, part);
    hipLaunchKernelGGL(k_bias_reduce, dim3(1), dim3(128), 0, st, part, cout, nchunk, gb);
}

// Adam (Kingma & Ba) on the FP32 master weights, then the BF16 copy
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, uint16_t* __restrict__ wbf, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        wbf[i] = f2bf(wi);
    }
}

void launch_adam(float* w, float* m, float* v, const float* g, uint16_t* wbf, int64_t n, float lr, float b1,
                 float b2, float eps, int64_t step, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(512), dim3(256), 0, st, w, m, v, g, wbf, n, lr, b1, b2, eps, c1, c2);
}

__global__ void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wbf, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        wbf[i] = f2bf(w[i]);
}

void launch_to_bf16(const float* w, uint16_t* wbf, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(512), dim3(256), 0, st, w, wbf, n);
}

// ------------------------------------------------------------ seed proposal
// Per event (one work-group): candidate bins are those whose logit exceeds
// logit(tau) (and, with nms, every one of their 8 neighbours; equal
// neighbours: the lower bin index wins); the best k_max by score (ties: lower
// index) become seeds at their bin centres, x0 = y0 = 0.  The event falls
// back to the lattice when its best logit is below logit(conf_min) or it has
// no candidate.  Both thresholds arrive as FP32 logits rounded from FP64.
constexpr int kCandCap = 4096;  // >= k_max; also the most strict maxima a 128 x 128 image can hold

// descending order of score, then ascending bin index, as an ascending u64 key;
// distinct bins give distinct keys, and every key is non-zero
__device__ __forceinline__ uint64_t cand_key(float v, int i)
{
    uint32_t b = __float_as_uint(v);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((uint64_t)b << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)i);
}

__device__ __forceinline__ bool is_cand(const float* __restrict__ z, int i, float v, float ltau, int nms)
{
    if (!(v > ltau)) return false;
    if (!nms) return true;
    const int r = i / kImg, c = i % kImg;
    for (int dr = -1; dr <= 1; ++dr)
        for (int dc = -1; dc <= 1; ++dc) {
            if (!dr && !dc) continue;
            const int rr = r + dr, cc = c + dc;
            if (rr < 0 || rr >= kImg || cc < 0 || cc >= kImg) continue;
            const int j = rr * kImg + cc;
            const float u = z[j];
            if (u > v || (u == v && j < i)) return false;
        }
    return true;
}

__global__ __launch_bounds__(256) void k_propose_select(ProposeArgs a)
{
    __shared__ uint64_t s_key[kCandCap];
    __shared__ int s_n, s_n2, s_rem;
    __shared__ uint64_t s_prefix;
    __shared__ uint32_t s_hist[256];
    __shared__ float s_best[256];
    const float ltau = a.ltau;
    for (int64_t e = blockIdx.x; e < a.n_events; e += gridDim.x) {
        const float* z = a.logits + e * kPix;
        if (threadIdx.x == 0) {
            s_n = 0;
            s_n2 = 0;
            s_rem = a.k_max;
            s_prefix = 0;
        }
        float best = -INFINITY;
        __syncthreads();
        // the logit reads of four positions go out together (the loop is
        // otherwise one dependent global read per position)
        constexpr int T = 256;  // the launch's work-group size
        static_assert(kPix % (4 * T) == 0, "whole groups of four positions per thread");
        for (int i0 = threadIdx.x; i0 < kPix; i0 += 4 * T) {
            float v4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v4[q] = z[i0 + q * T];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + q * T;
                best = fmaxf(best, v4[q]);
                if (!is_cand(z, i, v4[q], ltau, a.nms)) continue;
                const int slot = atomicAdd(&s_n, 1);
                if (slot < kCandCap) s_key[slot] = cand_key(v4[q], i);
            }
        }
        s_best[threadIdx.x] = best;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) s_best[threadIdx.x] = fmaxf(s_best[threadIdx.x], s_best[threadIdx.x + o]);
            __syncthreads();
        }
        int nc = s_n;
        if (nc > kCandCap) {
            // more candidates than fit (only without nms): radix-select the
            // k_max-th largest key, eight bits at a time from the top, then keep
            // exactly the keys at or above it
            for (int shift = 56; shift >= 0; shift -= 8) {
                for (int j = threadIdx.x; j < 256; j += blockDim.x) s_hist[j] = 0;
                __syncthreads();
                const uint64_t pfx = s_prefix;
                const uint64_t hm = shift == 56 ? 0ull : (~0ull << (shift + 8));
                for (int i = threadIdx.x; i < kPix; i += blockDim.x) {
                    const float v = z[i];
                    if (!is_cand(z, i, v, ltau, a.nms)) continue;
                    const uint64_t key = cand_key(v, i);
                    if ((key & hm) == pfx) atomicAdd(&s_hist[(key >> shift) & 255u], 1u);
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    int rem = s_rem;
                    for (int d = 255; d >= 0; --d) {
                        const int cnt = (int)s_hist[d];
                        if (cnt >= rem) {
                            s_prefix = pfx | ((uint64_t)d << shift);
                            break;
                        }
                        rem -= cnt;
                    }
                    s_rem = rem;
                }
                __syncthreads();
            }
            const uint64_t kth = s_prefix;
            for (int i = threadIdx.x; i < kPix; i += blockDim.x) {
                const float v = z[i];
                if (!is_cand(z, i, v, ltau, a.nms)) continue;
                const uint64_t key = cand_key(v, i);
                if (key >= kth) s_key[atomicAdd(&s_n2, 1)] = key;  // exactly k_max keys
            }
            __syncthreads();
            nc = a.k_max;
        }
        int np2 = 1;
        while (np2 < nc) np2 <<= 1;
        for (int i = nc + threadIdx.x; i < np2; i += blockDim.x) s_key[i] = 0;
        __syncthreads();
        for (int k = 2; k <= np2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < np2; i += blockDim.x) {
                    const int l = i ^ j;
                    if (l > i) {
                        const uint64_t x = s_key[i], y = s_key[l];
                        const bool desc = (i & k) == 0;
                        if (desc ? (x < y) : (x > y)) { s_key[i] = y; s_key[l] = x; }
                    }
                }
                __syncthreads();
            }
        const int keep = min(nc, a.k_max);
        // the kept bins are emitted in bin order (tx bin major): a wavefront's
        // seeds then sit in a narrow slope band, which keeps pruned passes short
        int kp2 = 1;
        while (kp2 < keep) kp2 <<= 1;
        for (int i = threadIdx.x; i < kp2; i += blockDim.x) {
            uint64_t v = ~0ull;
            if (i < keep) {
                const uint64_t key = s_key[i];
                v = ((uint64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull)) << 32) | (key >> 32);
            }
            s_key[i] = v;
        }
        __syncthreads();
        for (int k = 2; k <= kp2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < kp2; i += blockDim.x) {
                    const int l = i ^ j;
                    if (l > i) {
                        const uint64_t x = s_key[i], y = s_key[l];
                        const bool up = (i & k) == 0;
                        if (up ? (x > y) : (x < y)) { s_key[i] = y; s_key[l] = x; }
                    }
                }
                __syncthreads();
            }
        for (int i = threadIdx.x; i < keep; i += blockDim.x) {
            const uint64_t key = s_key[i];
            uint32_t b = (uint32_t)(key & 0xFFFFFFFFull);
            b = (b & 0x80000000u) ? (b & 0x7FFFFFFFu) : ~b;
            a.cand_score[e * a.k_max + i] = __uint_as_float(b);
            a.cand_pix[e * a.k_max + i] = (int32_t)(key >> 32);
        }
        if (threadIdx.x == 0) {
            a.confidence[e] = 1.0f / (1.0f + expf(-s_best[0]));
            const bool fb = !(s_best[0] >= a.lconf) || keep == 0;
            a.fallback[e] = fb ? 1 : 0;
            a.count[e] = fb ? a.lattice_n[0] * a.lattice_n[1] : keep;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_propose_offsets(ProposeArgs a)
{
    __shared__ int64_t s[1024];
    int64_t carry = 0;
    for (int64_t e0 = 0; e0 < a.n_events; e0 += 1024) {
        const int64_t e = e0 + threadIdx.x;
        const int64_t v = e < a.n_events ? a.count[e] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t add = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (e < a.n_events) a.seed_off[e] = carry + s[threadIdx.x] - v;
        const int64_t tot = s[1023];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) a.seed_off[a.n_events] = carry;
}

__global__ __launch_bounds__(256) void k_propose_write(ProposeArgs a)
{
    // coordinates come from host-formed tables: the bin centres (FP32 rounding
    // of lo + (i + 1/2) w formed in FP64) and the fallback lattice's centres
    for (int64_t e = blockIdx.x; e < a.n_events; e += gridDim.x) {
        double* out = a.seeds + a.seed_off[e] * 4;
        const int n = a.count[e];
        if (a.fallback[e]) {
            const int n0 = a.lattice_n[0], n1 = a.lattice_n[1];
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int i0 = i / n1, i1 = i % n1;
                out[4 * i + 0] = 0.0;
                out[4 * i + 1] = 0.0;
                out[4 * i + 2] = (double)a.lat_coord[i0];
                out[4 * i + 3] = (double)a.lat_coord[n0 + i1];
            }
        } else {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int pix = a.cand_pix[e * a.k_max + i];
                out[4 * i + 0] = 0.0;
                out[4 * i + 1] = 0.0;
                out[4 * i + 2] = (double)a.bin_centre[pix / kImg];
                out[4 * i + 3] = (double)a.bin_centre[pix % kImg];
            }
        }
    }
}

void launch_propose_select(const ProposeArgs& a, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>(a.n_events, 2048);
    hipLaunchKernelGGL(k_propose_select, dim3(grid), dim3(256), 0, st, a);
}

void launch_propose_offsets(const ProposeArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_propose_offsets, dim3(1), dim3(1024), 0, st, a);
}

void launch_propose_write(const ProposeArgs& a, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>(a.n_events, 2048);
    hipLaunchKernelGGL(k_propose_write, dim3(grid), dim3(256), 0, st, a);
}

// event_flags[e] |= 16 where the event's seeds came from the lattice fallback
__global__ __launch_bounds__(256) void k_flag_fallback(int32_t* __restrict__ ev_flags,
                                                       const int32_t* __restrict__ fallback, int64_t n_events)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_events;
         e += (int64_t)gridDim.x * blockDim.x)
        if (fallback[e]) ev_flags[e] |= 16;
}

void launch_flag_fallback(int32_t* ev_flags, const int32_t* fallback, int64_t n_events, hipStream_t st)
{
    if (n_events <= 0) return;
    const int grid = (int)std::min<int64_t>((n_events + 255) / 256, 1024);
    hipLaunchKernelGGL(k_flag_fallback, dim3(grid), dim3(256), 0, st, ev_flags, fallback, n_events);
}

// the same, with the event-flag array taken from the descriptor (out_ev_flags,
// may be NULL) so that a captured launch serves any caller array; skipped
// after a validation error (the outputs are not written then)
__global__ __launch_bounds__(256) void k_flag_fallback_desc(const Desc* __restrict__ d,
                                                            const int32_t* __restrict__ fallback)
{
    int32_t* ev_flags = d->out_ev_flags;
    if (!ev_flags || d->cnt->err) return;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < d->n_events;
         e += (int64_t)gridDim.x * blockDim.x)
        if (fallback[e]) ev_flags[e] |= 16;
}

size_t head_edge_floats(int64_t n_events) { return (size_t)n_events * (kImg / kCvRows) * kEdgeFloats; }

void launch_flag_fallback_desc(const Desc* d, const int32_t* fallback, int64_t n_events, hipStream_t st)
{
    if (n_events <= 0) return;
    const int grid = (int)std::min<int64_t>((n_events + 255) / 256, 1024);
    hipLaunchKernelGGL(k_flag_fallback_desc, dim3(grid), dim3(256), 0, st, d, fallback);
}

}  // namespace rt

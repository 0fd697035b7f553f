// The hot path: Eq. (1) with its gradient and Hessian, evaluated for many
// candidate lines against every hit of an event, and the multi-start
// truncated-Newton ascent built on it (Algorithm 1).
//
// Layout and work split (CDNA4, wave64):
//   * a work-group (4 waves) owns one event's hits in LDS and 4*64*C
//     candidate lines (C per lane, each wave its own 64*C);
//   * every lane walks the same hit (an LDS broadcast read), so the hit loop
//     is wave-uniform and the per-pair work is pure VALU: two residuals of two
//     subtractions each, one exp2 and six running sums; with few seeds per
//     event the ascent instead gives each seed 4 lanes, each over every 4th
//     hit (4 broadcast reads per wave), and adds their sums after each pass;
//   * hits are grouped by plane, where z is constant, so the per-pair sums are
//     P_e, P_x, P_y, P_xx, P_yy, P_xy and the z-moments are folded once per
//     plane into 16 accumulators (8 for meas_dim 1);
//   * events larger than the LDS tile are streamed through it tile by tile;
//   * the kernels are persistent: work-groups pull (event, seed block) items
//     from an atomic cursor over a longest-first list.
//
// Residuals: x reaches ~260 mm, where one FP32 ulp is already ~1.5e-5 mm,
// too coarse next to a 0.03 mm bandwidth, so the predicted position
// x0 + t z of a line on a plane is never rounded to one float.  Once per
// (line, plane) it is split exactly into s + l (s the rounded value, l its
// error, from the exact product error of an fma and the exact error of one
// addition); every hit of the plane then costs (x - s) - l, where x - s is
// exact whenever x lies within a factor 2 of s (every hit near the line), so
// the residual carries one rounding of its own size.  Both subtractions take
// VGPR operands only, which gfx950 issues at twice the rate of an fma with
// the plane's z in a scalar register.  The FP64 polish evaluates at an FP64
// theta split into two floats (hi + lo); the low words join l, so the
// gradient it solves with belongs to the FP64 point.
#include <algorithm>
#include <type_traits>

#include "rt_internal.h"

namespace rt {

constexpr float kLog2e = 1.44269504088896340736f;
// Lanes per seed of the split ascent (one candidate per lane, Newton steps):
// each of a seed's lanes walks every kSplitLanes-th hit of a plane segment.
// Work items with few seeds run with up to kMaxSplitLanes lanes per seed.
constexpr int kSplitLanes = 4;
constexpr int kMaxSplitLanes = 16;
// spare hit entries after the LDS tile: the meas_dim-2 hit loops read ahead
// of the segment they walk, up to index tile_hits + 2 * stride - 1 (split
// kernels: the line search walks with up to 64 lanes per trial point; the
// others: stride one).  The pad is part of the tile's LDS bytes, so it is
// kept as small as each shape allows: the dense ascent's tile is sized to fit
// three work-groups per CU.
constexpr int kTilePadSplit = 2 * kWave;
constexpr int kTilePad = 8;

template <int D>
struct Acc;  // number of accumulators
template <>
struct Acc<2> { static constexpr int N = 16; };
template <>
struct Acc<1> { static constexpr int N = 8; };

// Candidate line parameters held by a lane: offsets o[], slopes t[] per
// measured coordinate (meas_dim 1 uses index 0 only).
template <int C>
struct Cands {
    float o[C][2];
    float t[C][2];
};

// s + l = o + t z up to ~2^-48 relative (s = fl(o + t z)); with the polish's
// low words (ol, tl) added to l.
__device__ __forceinline__ void line_split(float o, float t, float z, float& s, float& l)
{
#pragma clang fp contract(off)  // s must be fl(p + o) for the error terms to be exact
    const float p = t * z;
    const float pe = __builtin_fmaf(t, z, -p);  // t z - p, exact
    s = p + o;
    const float bb = s - p;
    const float se = (p - (s - bb)) + (o - bb);  // p + o - s, exact
    l = pe + se;
}

__device__ __forceinline__ void line_split(float o, float t, float ol, float tl, float z, float& s, float& l)
{
    line_split(o, t, z, s, l);
    l += __builtin_fmaf(tl, z, ol);
}

// One plane segment [lo, hi) of LDS hits at plane position z.  QS > 1 (split):
// the wave's QS groups of 64 / QS lanes hold the same candidates and group g
// walks hits lo + g, lo + g + QS, ...; event_pass adds the groups' sums.
template <int D, int C, bool DERIV, bool DF, int QS = 1>
__device__ __forceinline__ void seg_accumulate(const float* __restrict__ s_hits, int lo, int hi,
                                               float z, const Cands<C>& c, const Cands<C>& cl,
                                               float nc, float (&acc)[C][Acc<D>::N])
{
    float pe[C], px[C], py[C], pxx[C], pyy[C], pxy[C];
    float sp[C][2], lp[C][2];  // the lines' positions on this plane, s + l
#pragma unroll
    for (int j = 0; j < C; ++j) {
        pe[j] = px[j] = py[j] = pxx[j] = pyy[j] = pxy[j] = 0.0f;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            if (DF) line_split(c.o[j][m], c.t[j][m], cl.o[j][m], cl.t[j][m], z, sp[j][m], lp[j][m]);
            else line_split(c.o[j][m], c.t[j][m], z, sp[j][m], lp[j][m]);
        }
    }
    if constexpr (D == 2) {
        const float2* h = reinterpret_cast<const float2*>(s_hits);
        auto pair = [&](const float2 v) {
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const float rx = (v.x - sp[j][0]) - lp[j][0];
                const float ry = (v.y - sp[j][1]) - lp[j][1];
                const float d2 = __builtin_fmaf(ry, ry, rx * rx);
                const float e = __builtin_amdgcn_exp2f(d2 * nc);
                pe[j] += e;
                if (DERIV) {
                    const float ex = e * rx;
                    const float ey = e * ry;
                    px[j] += ex;
                    py[j] += ey;
                    pxx[j] = __builtin_fmaf(ex, rx, pxx[j]);
                    pyy[j] = __builtin_fmaf(ey, ry, pyy[j]);
                    pxy[j] = __builtin_fmaf(ex, ry, pxy[j]);
                }
            }
        };
        // two hits per iteration; the next two are read from LDS while these
        // are processed.  The reads run up to 2 QS - 1 entries past the
        // segment: the LDS tile carries kTilePad (QS = 1) or kTilePadSplit
        // spare entries, so they stay inside it, and their values are never used.
        if constexpr (QS == 1) {
            float2 a = h[lo], b = h[lo + 1];
            int k = lo;
            for (; k + 1 < hi; k += 2) {
                const float2 na = h[k + 2], nb = h[k + 3];
                pair(a);
                pair(b);
                a = na;
                b = nb;
            }
            if (k < hi) pair(a);
        } else {
            const int k0 = lo + (int)(__lane_id() / (kWave / QS));
            float2 a = h[k0], b = h[k0 + QS];
            int k = k0;
            for (; k + QS < hi; k += 2 * QS) {
                const float2 na = h[k + 2 * QS], nb = h[k + 3 * QS];
                pair(a);
                pair(b);
                a = na;
                b = nb;
            }
            if (k < hi) pair(a);
        }
    } else {
        const int k0 = QS == 1 ? lo : lo + (int)(__lane_id() / (kWave / QS));
#pragma unroll 4
        for (int k = k0; k < hi; k += QS) {
            const float v = s_hits[k];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const float r = (v - sp[j][0]) - lp[j][0];
                const float e = __builtin_amdgcn_exp2f((r * r) * nc);
                pe[j] += e;
                if (DERIV) {
                    const float er = e * r;
                    px[j] += er;
                    pxx[j] = __builtin_fmaf(er, r, pxx[j]);
                }
            }
        }
    }
    const float z2 = z * z;
#pragma unroll
    for (int j = 0; j < C; ++j) {
        float* a = acc[j];
        a[0] += pe[j];
        if (DERIV) {
            a[1] = __builtin_fmaf(pe[j], z, a[1]);
            a[2] = __builtin_fmaf(pe[j], z2, a[2]);
            if constexpr (D == 2) {
                a[3] += px[j];
                a[4] = __builtin_fmaf(px[j], z, a[4]);
                a[5] += py[j];
                a[6] = __builtin_fmaf(py[j], z, a[6]);
                a[7] += pxx[j];
                a[8] = __builtin_fmaf(pxx[j], z, a[8]);
                a[9] = __builtin_fmaf(pxx[j], z2, a[9]);
                a[10] += pyy[j];
                a[11] = __builtin_fmaf(pyy[j], z, a[11]);
                a[12] = __builtin_fmaf(pyy[j], z2, a[12]);
                a[13] += pxy[j];
                a[14] = __builtin_fmaf(pxy[j], z, a[14]);
                a[15] = __builtin_fmaf(pxy[j], z2, a[15]);
            } else {
                a[3] += px[j];
                a[4] = __builtin_fmaf(px[j], z, a[4]);
                a[5] += pxx[j];
                a[6] = __builtin_fmaf(pxx[j], z, a[6]);
                a[7] = __builtin_fmaf(pxx[j], z2, a[7]);
            }
        }
    }
}

// Per-event context held by the work-group.
struct EventView {
    const float* g_hits;  // global staged hits of the event (first hit)
    int n;                // hits
    int P;
    bool resident;        // all hits already in LDS
    int tile_cap;
    bool prune;           // plane segments sorted by x: passes visit only each wave's x window
};

// ------------------------------------------------------------ pruning
// A pass may skip the hits of a plane whose x lies farther than
// w = sqrt(prune_u) sigma from the predicted x of every candidate the wave
// holds: each skipped term is below exp(-prune_u), so R changes by less than
// (hits) * exp(-prune_u) and the derivatives by the same factor times their
// polynomial weights.  The hits of a plane are sorted by x, the window is
// wave-uniform, and its index range comes from two rounds of 64 parallel
// probes (segments hold at most 4096 hits).
template <int D>
__device__ __forceinline__ float hit_key(const float* s_hits, int i)
{
    if constexpr (D == 2) return reinterpret_cast<const float2*>(s_hits)[i].x;
    else return s_hits[i];
}

// first index in [lo, hi) whose key is >= v (STRICT: > v); v wave-uniform,
// keys ascending, hi - lo <= 4096; every lane of the wave must call it
template <int D, bool STRICT>
__device__ __forceinline__ int wave_bound(const float* s_hits, int lo, int hi, float v)
{
    const int n = hi - lo;
    if (n <= 0) return lo;
    const int lane = threadIdx.x & (kWave - 1);
    const int step = (n + kWave - 1) / kWave;
    const int i1 = lo + lane * step;
    bool below = false;
    if (i1 < hi) {
        const float k = hit_key<D>(s_hits, i1);
        below = STRICT ? (k <= v) : (k < v);
    }
    const int c = __popcll(__ballot(below));
    if (c == 0) return lo;
    const int base = lo + (c - 1) * step + 1;
    const int end = min(hi, lo + c * step);
    const int i2 = base + lane;
    bool below2 = false;
    if (lane < step - 1 && i2 < end) {
        const float k = hit_key<D>(s_hits, i2);
        below2 = STRICT ? (k <= v) : (k < v);
    }
    return __builtin_amdgcn_readfirstlane(base + __popcll(__ballot(below2)));
}

// x window [xlo, xhi] of the wave's live candidates at plane z
template <int C>
__device__ __forceinline__ void wave_window(const Cands<C>& c, const bool* live, float z, float w, float& xlo,
                                            float& xhi)
{
    float mn = INFINITY, mx = -INFINITY;
#pragma unroll
    for (int j = 0; j < C; ++j) {
        if (live && !live[j]) continue;
        const float xc = __builtin_fmaf(c.t[j][0], z, c.o[j][0]);
        mn = fminf(mn, xc);
        mx = fmaxf(mx, xc);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, off, kWave));
        mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
    }
    xlo = mn - w;
    xhi = mx + w;
}

// the part [lo, hi) of a plane segment (tile-relative) inside the window
template <int D, int C>
__device__ __forceinline__ void prune_range(const float* s_hits, const Cands<C>& c, const bool* live, float z,
                                            float w, int& lo, int& hi)
{
    float xlo, xhi;
    wave_window<C>(c, live, z, w, xlo, xhi);
    const int a = wave_bound<D, false>(s_hits, lo, hi, xlo);
    const int b = wave_bound<D, true>(s_hits, lo, hi, xhi);
    lo = a;
    hi = max(a, b);
}

__device__ __forceinline__ float prune_width(const Desc* __restrict__ d, float nc)
{
    // nc = -log2(e) / sigma^2
    return sqrtf(d->prune_u * (-1.44269504088896340736f / nc));
}

// One pass over all of the event's hits for the lane's C candidates.
// Tiled events are streamed through LDS; the work-group must call this
// uniformly then (it contains barriers).
// `work` (wave-uniform) false: the wave holds no live candidate and only takes
// part in the tile loads and barriers; its sums stay zero.
template <int D, int C, bool DERIV, bool DF, bool PR = false, int QS = 1>
__device__ __forceinline__ void event_pass(const Desc* __restrict__ d, float* s_hits,
                                           const int* s_poff, const EventView& ev,
                                           const Cands<C>& c, const Cands<C>& cl, float nc,
                                           float (&acc)[C][Acc<D>::N], bool work = true,
                                           const bool* live = nullptr)
{
    const float pw = PR && ev.prune ? prune_width(d, nc) : 0.0f;
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
        for (int a = 0; a < Acc<D>::N; ++a) acc[j][a] = 0.0f;
    for (int t0 = 0; t0 < ev.n; t0 += ev.tile_cap) {
        const int t1 = min(ev.n, t0 + ev.tile_cap);
        if (!ev.resident) {
            __syncthreads();
            if (D == 2) {
                const float2* src = reinterpret_cast<const float2*>(ev.g_hits) + t0;
                float2* dst = reinterpret_cast<float2*>(s_hits);
                for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) dst[i] = src[i];
            } else {
                for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) s_hits[i] = ev.g_hits[t0 + i];
            }
            __syncthreads();
        }
        if (!work) continue;
        for (int p = 0; p < ev.P; ++p) {
            // LDS values are the same in every lane: keep the loop bounds scalar
            int lo = __builtin_amdgcn_readfirstlane(max(s_poff[p], t0)) - t0;
            int hi = __builtin_amdgcn_readfirstlane(min(s_poff[p + 1], t1)) - t0;
            if (lo >= hi) continue;
            const float z = d->plane_z[p];
            if constexpr (PR) {
                if (ev.prune) {
                    prune_range<D, C>(s_hits, c, live, z, pw, lo, hi);
                    if (lo >= hi) continue;
                }
            }
            seg_accumulate<D, C, DERIV, DF, QS>(s_hits, lo, hi, z, c, cl, nc, acc);
        }
    }
    if constexpr (QS > 1) {
        // butterfly over the groups: at each level one lane adds a + b and its
        // partner b + a, so every lane of a seed ends with the same bits
#pragma unroll
        for (int m = kWave / 2; m >= kWave / QS; m >>= 1)
#pragma unroll
            for (int j = 0; j < C; ++j)
#pragma unroll
                for (int a = 0; a < Acc<D>::N; ++a) acc[j][a] += __shfl_xor(acc[j][a], m);
    }
}

// R only, one candidate per thread, over the hits of every plane segment whose
// index within the segment is congruent to `part` modulo `parts` (threads of a
// wave may hold different parts: hit reads are then per lane).  The per-pair
// arithmetic is seg_accumulate's; per-plane sums are added in plane order.
// Same barrier rule as event_pass.
template <int D, bool PR = false>
__device__ __forceinline__ float event_pass_split(const Desc* __restrict__ d, float* s_hits, const int* s_poff,
                                                  const EventView& ev, const float* th, float nc, int part,
                                                  int parts, bool live = true)
{
    float R = 0.0f;
    const float pw = PR && ev.prune ? prune_width(d, nc) : 0.0f;
    // the window of every point the wave holds (each wave holds all of them)
    Cands<1> wc;
    if constexpr (D == 2) { wc.o[0][0] = th[0]; wc.t[0][0] = th[2]; }
    else { wc.o[0][0] = th[0]; wc.t[0][0] = th[1]; }
    const bool wl[1] = {live};
    for (int t0 = 0; t0 < ev.n; t0 += ev.tile_cap) {
        const int t1 = min(ev.n, t0 + ev.tile_cap);
        if (!ev.resident) {
            __syncthreads();
            if (D == 2) {
                const float2* src = reinterpret_cast<const float2*>(ev.g_hits) + t0;
                float2* dst = reinterpret_cast<float2*>(s_hits);
                for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) dst[i] = src[i];
            } else {
                for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) s_hits[i] = ev.g_hits[t0 + i];
            }
            __syncthreads();
        }
        for (int p = 0; p < ev.P; ++p) {
            int lo = __builtin_amdgcn_readfirstlane(max(s_poff[p], t0)) - t0;
            int hi = __builtin_amdgcn_readfirstlane(min(s_poff[p + 1], t1)) - t0;
            if (lo >= hi) continue;
            const float z = d->plane_z[p];
            if constexpr (PR) {
                if (ev.prune) {
                    prune_range<D, 1>(s_hits, wc, wl, z, pw, lo, hi);
                    if (lo >= hi) continue;
                }
            }
            float pe = 0.0f;
            // two hits per iteration, the next two read while these are summed;
            // indices are clamped to the segment, so every read is in bounds
            const int last = hi - 1;
            int k = lo + part;
            if constexpr (D == 2) {
                const float2* h = reinterpret_cast<const float2*>(s_hits);
                float sx, lx, sy, ly;
                line_split(th[0], th[2], z, sx, lx);
                line_split(th[1], th[3], z, sy, ly);
                auto term = [&](const float2 v) {
                    const float rx = (v.x - sx) - lx;
                    const float ry = (v.y - sy) - ly;
                    return __builtin_amdgcn_exp2f(__builtin_fmaf(ry, ry, rx * rx) * nc);
                };
                float2 a = h[min(k, last)], b = h[min(k + parts, last)];
                for (; k <= last; k += 2 * parts) {
                    const float2 na = h[min(k + 2 * parts, last)], nb = h[min(k + 3 * parts, last)];
                    pe += term(a);
                    if (k + parts <= last) pe += term(b);
                    a = na;
                    b = nb;
                }
            } else {
                float sx, lx;
                line_split(th[0], th[1], z, sx, lx);
                auto term = [&](const float v) {
                    const float r = (v - sx) - lx;
                    return __builtin_amdgcn_exp2f((r * r) * nc);
                };
                float a = s_hits[min(k, last)], b = s_hits[min(k + parts, last)];
                for (; k <= last; k += 2 * parts) {
                    const float na = s_hits[min(k + 2 * parts, last)], nb = s_hits[min(k + 3 * parts, last)];
                    pe += term(a);
                    if (k + parts <= last) pe += term(b);
                    a = na;
                    b = nb;
                }
            }
            R += pe;
        }
    }
    return R;
}

// R-only pass over part `part` of `parts` of every plane segment (the waves of a
// work-group split the hits; their partial sums are added afterwards in a
// fixed order).  Same barrier rule as event_pass.
template <int D, int C, bool PR = false>
__device__ __forceinline__ void event_pass_part(const Desc* __restrict__ d, float* s_hits,
                                                const int* s_poff, const EventView& ev,
                                                const Cands<C>& c, float nc, int part, int parts,
                                                float (&acc)[C][Acc<D>::N], const bool* live = nullptr)
{
    const Cands<C> zero_c = {};
    const float pw = PR && ev.prune ? prune_width(d, nc) : 0.0f;
#pragma unroll
    for (int j = 0; j < C; ++j) acc[j][0] = 0.0f;
    for (int t0 = 0; t0 < ev.n; t0 += ev.tile_cap) {
        const int t1 = min(ev.n, t0 + ev.tile_cap);
        if (!ev.resident) {
            __syncthreads();
            if (D == 2) {
                const float2* src = reinterpret_cast<const float2*>(ev.g_hits) + t0;
                float2* dst = reinterpret_cast<float2*>(s_hits);
                for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) dst[i] = src[i];
            } else {
                for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) s_hits[i] = ev.g_hits[t0 + i];
            }
            __syncthreads();
        }
        for (int p = 0; p < ev.P; ++p) {
            int lo = __builtin_amdgcn_readfirstlane(max(s_poff[p], t0)) - t0;
            int hi = __builtin_amdgcn_readfirstlane(min(s_poff[p + 1], t1)) - t0;
            if (lo >= hi) continue;
            const float z = d->plane_z[p];
            if constexpr (PR) {
                if (ev.prune) {
                    prune_range<D, C>(s_hits, c, live, z, pw, lo, hi);
                    if (lo >= hi) continue;
                }
            }
            const int len = hi - lo;
            const int a = lo + (len * part) / parts;
            const int b = lo + (len * (part + 1)) / parts;
            if (a >= b) continue;
            seg_accumulate<D, C, false, false>(s_hits, a, b, z, c, zero_c, nc, acc);
        }
    }
}

// Gradient and Hessian from the accumulators (formulas of Eq. (1)
// differentiated; theta order (x0, y0, tx, ty) or (x0, tx)).  Full matrix.
template <int D, typename T>
__device__ __forceinline__ void grad_hess(const float* a, float sigma, T* g, T (*H)[2 * D])
{
    const T s2 = (T)sigma * (T)sigma;
    const T two = (T)2 / s2;
    const T four = (T)4 / (s2 * s2);
    if constexpr (D == 2) {
        g[0] = two * (T)a[3];
        g[1] = two * (T)a[5];
        g[2] = two * (T)a[4];
        g[3] = two * (T)a[6];
        H[0][0] = four * (T)a[7] - two * (T)a[0];
        H[0][1] = four * (T)a[13];
        H[0][2] = four * (T)a[8] - two * (T)a[1];
        H[0][3] = four * (T)a[14];
        H[1][1] = four * (T)a[10] - two * (T)a[0];
        H[1][2] = four * (T)a[14];
        H[1][3] = four * (T)a[11] - two * (T)a[1];
        H[2][2] = four * (T)a[9] - two * (T)a[2];
        H[2][3] = four * (T)a[15];
        H[3][3] = four * (T)a[12] - two * (T)a[2];
    } else {
        g[0] = two * (T)a[3];
        g[1] = two * (T)a[4];
        H[0][0] = four * (T)a[5] - two * (T)a[0];
        H[0][1] = four * (T)a[6] - two * (T)a[1];
        H[1][1] = four * (T)a[7] - two * (T)a[2];
    }
#pragma unroll
    for (int i = 0; i < 2 * D; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) H[i][j] = H[j][i];
}

// Truncated-Newton direction for maximising R in scaled coordinates
// (scaled = ds * theta): conjugate gradients on (-H~) p~ = g~ from zero, at
// most N iterations, stopping at a residual below 1e-4 |g~|; a non-positive
// curvature on the first direction gives a steepest-ascent step of one
// bandwidth, on a later one the current iterate.  The scaled step is capped
// at cap*sigma.  Returns the unscaled direction.
template <int N>
__device__ __forceinline__ void newton_cg(const float* g, const float (*H)[N], const float* ds,
                                          float sigma, float cap, float* p, float& pn, bool& neg)
{
    float b[N], A[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = g[i] / ds[i];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) A[i][j] = -H[i][j] / (ds[i] * ds[j]);
    float bb = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) bb = __builtin_fmaf(b[i], b[i], bb);
    const float bn = sqrtf(bb);
    float q[N];
#pragma unroll
    for (int i = 0; i < N; ++i) q[i] = 0.0f;
    neg = false;
    if (bn > 0.0f) {
        const float tol = 1e-4f * bn;
        float x[N], r[N], dv[N];
#pragma unroll
        for (int i = 0; i < N; ++i) { x[i] = 0.0f; r[i] = b[i]; dv[i] = b[i]; }
        bool done = false;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (!done) {
                float Ad[N], dAd = 0.0f, rr = 0.0f;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    float s = 0.0f;
#pragma unroll
                    for (int j = 0; j < N; ++j) s = __builtin_fmaf(A[i][j], dv[j], s);
                    Ad[i] = s;
                }
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    dAd = __builtin_fmaf(dv[i], Ad[i], dAd);
                    rr = __builtin_fmaf(r[i], r[i], rr);
                }
                if (!(dAd > 0.0f)) {
                    neg = true;
                    if (k == 0) {
#pragma unroll
                        for (int i = 0; i < N; ++i) q[i] = sigma * (b[i] / bn);
                    } else {
#pragma unroll
                        for (int i = 0; i < N; ++i) q[i] = x[i];
                    }
                    done = true;
                } else {
                    const float alpha = rr / dAd;
                    float rn = 0.0f;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        x[i] = __builtin_fmaf(alpha, dv[i], x[i]);
                        r[i] = __builtin_fmaf(-alpha, Ad[i], r[i]);
                        rn = __builtin_fmaf(r[i], r[i], rn);
                    }
                    if (sqrtf(rn) < tol) {
#pragma unroll
                        for (int i = 0; i < N; ++i) q[i] = x[i];
                        done = true;
                    } else {
                        const float beta = rn / rr;
#pragma unroll
                        for (int i = 0; i < N; ++i) dv[i] = __builtin_fmaf(beta, dv[i], r[i]);
                    }
                }
            }
        }
        if (!done) {
#pragma unroll
            for (int i = 0; i < N; ++i) q[i] = x[i];
        }
    }
    float qq = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) qq = __builtin_fmaf(q[i], q[i], qq);
    pn = sqrtf(qq);
    const float lim = cap * sigma;
    if (pn > lim) {
        const float s = lim / pn;
#pragma unroll
        for (int i = 0; i < N; ++i) q[i] *= s;
        pn = lim;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = q[i] / ds[i];
}

// FP64 Cholesky solve of A x = b (N <= 4); false when A is not positive definite.
template <int N>
__device__ __forceinline__ bool chol_solve(const double (*A)[N], const double* b, double* x)
{
    double L[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) L[i][j] = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0)) { ok = false; s = 1.0; }
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    double y[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < N; ++k) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return ok;
}

// theta (x0, y0, tx, ty) / (x0, tx) <-> lane candidate slots
template <int D, int C>
__device__ __forceinline__ void set_cand(Cands<C>& c, int j, const float* th)
{
    if constexpr (D == 2) { c.o[j][0] = th[0]; c.o[j][1] = th[1]; c.t[j][0] = th[2]; c.t[j][1] = th[3]; }
    else { c.o[j][0] = th[0]; c.t[j][0] = th[1]; c.o[j][1] = 0.0f; c.t[j][1] = 0.0f; }
}

__device__ __forceinline__ bool wg_or(bool v, bool resident)
{
    // resident events have no barriers inside a pass: waves may iterate on their own
    if (resident) return __any(v) != 0;
    return __syncthreads_or(v) != 0;
}

// Load the event's plane offsets (event-relative) and, if it fits, its hits.
// With parts > 1 the view is part `part` of the event's hits (a contiguous
// range across planes; plane segments are clipped to it).
__device__ __forceinline__ EventView begin_event(const Desc* __restrict__ d, int e, float* s_hits,
                                                 int* s_poff, int tile_cap, int part = 0, int parts = 1)
{
    const int P = d->n_planes;
    const int32_t* po = d->plane_off + (int64_t)e * (P + 1);
    const int n_all = d->ev_nhits[e];
    const int h0 = (int)((int64_t)n_all * part / parts), h1 = (int)((int64_t)n_all * (part + 1) / parts);
    const int base = po[0] + h0;
    EventView ev;
    ev.P = P;
    ev.n = h1 - h0;
    ev.g_hits = d->hits + (int64_t)base * d->meas_dim;
    ev.tile_cap = tile_cap;
    ev.resident = ev.n <= tile_cap;
    ev.prune = d->prune_u > 0.0f && parts == 1 && d->ev_sorted != nullptr && d->ev_sorted[e] != 0;
    if ((int)threadIdx.x <= P) s_poff[threadIdx.x] = min(max(po[threadIdx.x] - base, 0), h1 - h0);
    if (ev.resident) {
        if (d->meas_dim == 2) {
            const float2* src = reinterpret_cast<const float2*>(ev.g_hits);
            float2* dst = reinterpret_cast<float2*>(s_hits);
            for (int i = threadIdx.x; i < ev.n; i += blockDim.x) dst[i] = src[i];
        } else {
            for (int i = threadIdx.x; i < ev.n; i += blockDim.x) s_hits[i] = ev.g_hits[i];
        }
    }
    __syncthreads();
    return ev;
}

// R only at one line per lane group over a resident event: the point of lane
// l is point l % (64 / L), and its L lanes walk every L-th hit of each plane
// segment with the passes' own hit loop (R only), then a butterfly over the
// L lanes adds their sums in a fixed order.  Reads run up to 2 L - 1 entries
// past a segment (the split tile's spare entries cover L = 64).
template <int D, int L>
__device__ __forceinline__ float group_response(const Desc* __restrict__ d, const float* s_hits, const int* s_poff,
                                                const EventView& ev, const float* th, float nc)
{
    static_assert(2 * L <= kTilePadSplit, "the read-ahead stays inside the tile's spare entries");
    Cands<1> c;
    set_cand<D, 1>(c, 0, th);
    const Cands<1> zero_c = {};
    float acc[1][Acc<D>::N];
#pragma unroll
    for (int a = 0; a < Acc<D>::N; ++a) acc[0][a] = 0.0f;
    for (int p = 0; p < ev.P; ++p) {
        const int lo = __builtin_amdgcn_readfirstlane(s_poff[p]);
        const int hi = __builtin_amdgcn_readfirstlane(s_poff[p + 1]);
        if (lo >= hi) continue;
        seg_accumulate<D, 1, false, false, L>(s_hits, lo, hi, d->plane_z[p], c, zero_c, nc, acc);
    }
    float r = acc[0][0];
#pragma unroll
    for (int m = kWave / 2; m >= kWave / L; m >>= 1) r += __shfl_xor(r, m);
    return r;
}

// Backtracking line search of one wave's seeds, wave-local (no work-group
// barrier), for the split ascent on a resident event.  The QS lanes of a seed
// hold identical state.  Each round takes the wave's m pending seeds (by their
// owner lanes), gives each trial point L = 64 / m lanes (rounded down to a
// power of two), which walk its hits as a pass does (group_response); a
// butterfly over the L lanes adds their parts in a fixed order.  Every seed either accepts,
// halves its step or stalls in a round, so at most ls_trials rounds run.
// Returns the pair evaluations of the wave (counted once, in lane 0).
template <int D, int QS>
__device__ __forceinline__ uint64_t wave_line_search(const Desc* __restrict__ d, const float* s_hits,
                                                     const int* s_poff, const EventView& ev,
                                                     float (&th)[2 * D], const float (&p)[2 * D], float Rc,
                                                     float gp, bool& pend, int& nre, int& flags, float nc)
{
    constexpr int NP = 2 * D;
    constexpr int SL = kWave / QS;
    const int lane = (int)__lane_id();
    const int slane = lane & (SL - 1);
    const bool owner = lane < SL;
    float alpha = 1.0f;
    int trial = 0;
    uint64_t pairs = 0;
    for (;;) {
        const uint64_t bal = __ballot(pend && owner);
        const int m = __popcll(bal);
        if (m == 0) break;
        int L = kWave;
        while (L * m > kWave) L >>= 1;
        const int q = lane & (kWave / L - 1);  // this lane's point
        const bool qlive = q < m;
        // owner lane of point q: the q-th set bit of bal
        uint64_t b = bal;
        for (int i = 0; i < q && i < 16; ++i) b &= b - 1;
        const int src = qlive ? __builtin_ctzll(b) : 0;
        float tt[NP], tq[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            tt[a] = __builtin_fmaf(alpha, p[a], th[a]);
            tq[a] = __shfl(tt[a], src);
        }
        // lanes of points past m evaluate point 0's line again (not read)
        float Rq;
        switch (L) {
        case 64: Rq = group_response<D, 64>(d, s_hits, s_poff, ev, tq, nc); break;
        case 32: Rq = group_response<D, 32>(d, s_hits, s_poff, ev, tq, nc); break;
        case 16: Rq = group_response<D, 16>(d, s_hits, s_poff, ev, tq, nc); break;
        case 8: Rq = group_response<D, 8>(d, s_hits, s_poff, ev, tq, nc); break;
        default: Rq = group_response<D, 4>(d, s_hits, s_poff, ev, tq, nc); break;
        }
        // the seed's lanes read the sum of its point (point r sits in lane r)
        const int rank = __popcll(bal & ((1ull << slane) - 1ull));
        const float Rt = __shfl(Rq, rank);
        pairs += (uint64_t)m * (uint64_t)ev.n;
        if (pend) {
            ++nre;
            if (Rt >= Rc + d->armijo_c1 * alpha * gp) {
#pragma unroll
                for (int a = 0; a < NP; ++a) th[a] = tt[a];
                pend = false;
            } else if (++trial >= d->ls_trials) {
                pend = false;
                flags |= RETINA_STALLED;
            } else {
                alpha *= 0.5f;
            }
        }
    }
    return pairs;
}

// ------------------------------------------------------------------ ascent
// Lattice point i of an event (dimension 0 slow): D = 2 gives (0, 0, tx, ty),
// D = 1 gives (x0, tx) with tx along dimension 0.  The coordinates come from
// the descriptor's table (formed on the host).
template <int D>
__device__ __forceinline__ void lattice_point(const Desc* __restrict__ d, int i, float* th)
{
    const int n1 = d->lattice_n[1];
    const int i0 = i / n1, i1 = i % n1;
    const float v0 = d->lat_coord[i0];
    const float v1 = d->lat_coord[d->lattice_n[0] + i1];
    if constexpr (D == 2) { th[0] = 0.0f; th[1] = 0.0f; th[2] = v0; th[3] = v1; }
    else { th[0] = v1; th[1] = v0; }
}

// Update rules of the inner loop (U): 0 truncated Newton, 1 normalised
// gradient, 2 BFGS.  The rule is a template parameter so that the default
// Newton kernels carry no quasi-Newton state.
// QS > 1 (split, one candidate per lane, Newton): QS lane groups of a wave
// hold the same 64 / QS seeds and share every pass's hits, so a work item of
// 256 / QS seeds keeps all four waves busy with an event of few seeds; the
// groups' results are identical bit for bit, and the first group alone
// queues line-search points and writes results.
template <int D, int C, int U = 0, bool PR = false, int QS = 1>
__global__ __launch_bounds__(kBlock) void k_ascent(const Desc* __restrict__ d, int tile_cap)
{
    static_assert(QS == 1 || (C == 1 && U == 0), "split: one candidate per lane, Newton steps");
    constexpr int NP = 2 * D;
    constexpr int NA = Acc<D>::N;
    // dynamic LDS follows the static arrays: declared float4 so it starts 16-byte
    // aligned (the (x, y) hit pairs are read with 8-byte LDS loads)
    extern __shared__ float4 s_dyn[];
    float* s_hits = reinterpret_cast<float*>(s_dyn);
    __shared__ int s_poff[kMaxPlanes + 1];
    __shared__ int s_item;
    constexpr int kNW = kBlock / kWave;
    __shared__ int s_wcnt[C * kNW];         // line-search list: pending points per (slot j, wave),
    __shared__ float s_lth[kBlock * C][4];  // the points, then their responses (slot 0)
    __shared__ float s_red[kBlock];         // partial responses of a line-search round
    if (d->cnt->err) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // scalar: same in every lane
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t n_items = d->cnt->n_items;
    const int n_steps = d->n_sigma + d->n_final_steps;
    const float zr = d->z_ref;
    float ds[NP];
    if constexpr (D == 2) { ds[0] = 1.0f; ds[1] = 1.0f; ds[2] = zr; ds[3] = zr; }
    else { ds[0] = 1.0f; ds[1] = zr; }
    const Cands<C> zero_c = {};

    // this work-group's XCD queue first, then the others (work stealing at the end)
    const int xq = (int)(blockIdx.x % kXcds);
    (void)n_items;
    for (;;) {
        if (threadIdx.x == 0) {
            int found = -1;
            for (int k = 0; k < kXcds && found < 0; ++k) {
                const int q = (xq + k) % kXcds;
                const int64_t q0 = d->cnt->xq_start[q], nq = d->cnt->xq_start[q + 1] - q0;
                if (nq <= 0 || (int64_t)__hip_atomic_load(&d->cnt->xq_cursor[q][0], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT) >= nq)
                    continue;
                const uint32_t cidx = atomicAdd(&d->cnt->xq_cursor[q][0], 1u);
                if ((int64_t)cidx < nq) found = (int)(q0 + cidx);
            }
            s_item = found;
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item < 0) break;
        const int2 it0 = d->items[item];
        // seeds [it.y, it.y + isz) of event it.x; a negative block is a half block
        const int isz = it0.y < 0 ? d->seeds_per_item / 2 : d->seeds_per_item;
        const int2 it = make_int2(it0.x, (it0.y < 0 ? ~it0.y : it0.y) * isz);
        const int e = __builtin_amdgcn_readfirstlane(it.x);
        const EventView ev = begin_event(d, e, s_hits, s_poff, tile_cap);
        const int64_t sbase = d->seed_off[e];
        const int ns = (int)(d->seed_off[e + 1] - sbase);
        // lanes per seed for this item: a half item (an event's part-filled
        // seeds, at most 32) spreads its seeds over all four waves with 8 or
        // 16 lanes each (every pass then walks the hits in fewer strides), so
        // that it costs less than a full one
        auto item_body = [&](auto qtag) {
            constexpr int QS2 = decltype(qtag)::value;
            constexpr int SL2 = kWave / QS2;  // seeds per wave and candidate slot
            const int slane2 = lane & (SL2 - 1);  // the lane's seed within the wave's slot
            const bool owner2 = lane < SL2;       // queues line-search points, writes the results

            // seeds
            float th[C][NP];
            bool active[C];
            int flags[C], nre[C];
            // BFGS state per candidate (scaled coordinates): inverse-Hessian model
            // of -R, the previous step's scaled gradient and its accepted step
            constexpr int CQ = U == 2 ? C : 1;
            float Bq[CQ][NP][NP], bq[CQ][NP], sq[CQ][NP];
            float sig_prev = 0.0f;
    #pragma unroll
            for (int j = 0; j < C; ++j) {
                const int sj = it.y + (wave * C + j) * SL2 + slane2;
                active[j] = sj < ns && sj < it.y + isz;
                flags[j] = 0;
                nre[j] = 0;
                const int sjc = active[j] ? sj : 0;
                if (d->seed_mode == RETINA_SEED_EXPLICIT) {
                    const double* s = d->in_seeds + (sbase + sjc) * NP;
                    bool finite = true;
    #pragma unroll
                    for (int a = 0; a < NP; ++a) {
                        th[j][a] = active[j] ? (float)s[a] : 0.0f;
                        finite = finite && isfinite(th[j][a]);
                    }
                    if (!finite) {
                        // device-memory seeds are validated here: the call fails
                        // (no output is written) and the seed stays out of the passes
                        atomicOr(&d->cnt->err, kErrSeedVal);
                        active[j] = false;
    #pragma unroll
                        for (int a = 0; a < NP; ++a) th[j][a] = 0.0f;
                    }
                } else {
                    lattice_point<D>(d, sjc, th[j]);
                }
            }

            // waves without a live seed skip the arithmetic of every pass
            bool any_active = false;
    #pragma unroll
            for (int j = 0; j < C; ++j) any_active = any_active || active[j];
            const bool wave_work = __builtin_amdgcn_readfirstlane((int)(__any(any_active) != 0)) != 0;
            uint64_t ls_pairs = 0;  // executed line-search pair evaluations (same in every thread)
            uint64_t wls_pairs = 0; // ... of the wave-local searches (this wave's, in every lane)
            for (int s = 0; s < n_steps; ++s) {
                const float sig = s < d->n_sigma ? d->sigma[s] : d->sigma_final;
                const float nc = -kLog2e / (sig * sig);
                Cands<C> c;
    #pragma unroll
                for (int j = 0; j < C; ++j) set_cand<D, C>(c, j, th[j]);
                float acc[C][NA];
                event_pass<D, C, true, false, PR, QS2>(d, s_hits, s_poff, ev, c, zero_c, nc, acc, wave_work, active);
                float p[C][NP], Rc[C], gp[C], alpha[C];
                bool pend[C];
                int trial[C];
                const bool slope_only = D == 2 && s < d->n_slope_steps;
    #pragma unroll
                for (int j = 0; j < C; ++j) {
                    float g[NP], H[NP][NP];
                    grad_hess<D, float>(acc[j], sig, g, H);
                    float pn;
                    bool neg;
                    if constexpr (U != 0) {
                        // scaled gradient (offset components zero while they are held)
                        float b[NP], q[NP], bb = 0.0f;
    #pragma unroll
                        for (int a = 0; a < NP; ++a) b[a] = (D == 2 && slope_only && a < 2) ? 0.0f : g[a] / ds[a];
    #pragma unroll
                        for (int a = 0; a < NP; ++a) bb = __builtin_fmaf(b[a], b[a], bb);
                        const float bn = sqrtf(bb);
                        if constexpr (U == 1) {
    #pragma unroll
                            for (int a = 0; a < NP; ++a) q[a] = bn > 0.0f ? sig * (b[a] / bn) : 0.0f;
                        } else {
                            float (&B)[NP][NP] = Bq[U == 2 ? j : 0];
                            if (s == 0 || sig != sig_prev) {
                                // (re)start: the normalised gradient step of one bandwidth
    #pragma unroll
                                for (int a = 0; a < NP; ++a)
    #pragma unroll
                                    for (int c2 = 0; c2 < NP; ++c2) B[a][c2] = a == c2 ? (bn > 0.0f ? sig / bn : 0.0f) : 0.0f;
                            } else {
                                // BFGS with y = -(b - b_prev) (gradient change of -R) and
                                // the accepted step, in the expanded form
                                // B + ((s.y + y.B.y) / (s.y)^2) s s^T - (B y s^T + s y^T B) / s.y
                                float y[NP], sy = 0.0f;
    #pragma unroll
                                for (int a = 0; a < NP; ++a) {
                                    y[a] = bq[U == 2 ? j : 0][a] - b[a];
                                    sy = __builtin_fmaf(sq[U == 2 ? j : 0][a], y[a], sy);
                                }
                                if (sy > 0.0f) {
                                    float By[NP], yBy = 0.0f;
    #pragma unroll
                                    for (int a = 0; a < NP; ++a) {
                                        float v = 0.0f;
    #pragma unroll
                                        for (int c2 = 0; c2 < NP; ++c2) v = __builtin_fmaf(B[a][c2], y[c2], v);
                                        By[a] = v;
                                        yBy = __builtin_fmaf(y[a], v, yBy);
                                    }
                                    const float inv = 1.0f / sy;
                                    const float cs = (sy + yBy) * inv * inv;
                                    const float* sv = sq[U == 2 ? j : 0];
    #pragma unroll
                                    for (int a = 0; a < NP; ++a)
    #pragma unroll
                                        for (int c2 = 0; c2 < NP; ++c2)
                                            B[a][c2] += cs * sv[a] * sv[c2] - (By[a] * sv[c2] + sv[a] * By[c2]) * inv;
                                }
                            }
    #pragma unroll
                            for (int a = 0; a < NP; ++a) {
                                float v = 0.0f;
    #pragma unroll
                                for (int c2 = 0; c2 < NP; ++c2) v = __builtin_fmaf(B[a][c2], b[c2], v);
                                q[a] = v;
                                bq[U == 2 ? j : 0][a] = b[a];
                                sq[U == 2 ? j : 0][a] = 0.0f;
                            }
                        }
                        float qq = 0.0f;
    #pragma unroll
                        for (int a = 0; a < NP; ++a) qq = __builtin_fmaf(q[a], q[a], qq);
                        pn = sqrtf(qq);
                        const float lim = d->step_cap * sig;
                        if (pn > lim) {
                            const float sc = lim / pn;
    #pragma unroll
                            for (int a = 0; a < NP; ++a) q[a] *= sc;
                            pn = lim;
                        }
    #pragma unroll
                        for (int a = 0; a < NP; ++a) p[j][a] = q[a] / ds[a];
                        neg = false;
                    } else if constexpr (D == 2) {
                        if (slope_only) {
                            const float gs[2] = {g[2], g[3]};
                            const float Hs[2][2] = {{H[2][2], H[2][3]}, {H[3][2], H[3][3]}};
                            const float dss[2] = {ds[2], ds[3]};
                            float ps[2];
                            newton_cg<2>(gs, Hs, dss, sig, d->step_cap, ps, pn, neg);
                            p[j][0] = 0.0f; p[j][1] = 0.0f; p[j][2] = ps[0]; p[j][3] = ps[1];
                        } else {
                            newton_cg<NP>(g, H, ds, sig, d->step_cap, p[j], pn, neg);
                        }
                    } else {
                        newton_cg<NP>(g, H, ds, sig, d->step_cap, p[j], pn, neg);
                    }
                    if (neg) flags[j] |= RETINA_NEGCURV;
                    Rc[j] = acc[j][0];
                    float dot = 0.0f;
    #pragma unroll
                    for (int a = 0; a < NP; ++a) dot = __builtin_fmaf(g[a], p[j][a], dot);
                    gp[j] = dot;
                    alpha[j] = 1.0f;
                    trial[j] = 0;
                    if (!active[j]) {
                        pend[j] = false;  // an empty slot never searches
                    } else if (!neg && pn <= d->small_step * sig) {
    #pragma unroll
                        for (int a = 0; a < NP; ++a) th[j][a] += p[j][a];
                        if constexpr (U == 2) {
    #pragma unroll
                            for (int a = 0; a < NP; ++a) sq[j][a] = ds[a] * p[j][a];
                        }
                        pend[j] = false;
                    } else {
                        pend[j] = true;
                    }
                }
                sig_prev = sig;
                if constexpr (QS2 > 1 && !PR) {
                    if (ev.resident) {
                        // every hit in LDS: each wave searches for its own seeds
                        wls_pairs += wave_line_search<D, QS2>(d, s_hits, s_poff, ev, th[0], p[0], Rc[0], gp[0],
                                                             pend[0], nre[0], flags[0], nc);
                        continue;
                    }
                }
                // Backtracking line search.  Each round gathers the work-group's
                // pending trial points into an LDS list and evaluates R only for
                // those.  One candidate per lane and up to 64 pending points: the
                // 256 threads split into 256 / P parts per point (P = the count
                // rounded up to a power of two), each summing R over every
                // (256 / P)-th hit of each plane segment.  Otherwise: rounds of
                // 64 * C points per wave, every wave over its quarter of each plane
                // segment (C candidates per lane share each hit read; measured
                // faster for C = 2 even when few points are pending).  Partial sums
                // are added in a fixed order.  The list is in (slot j, wave, lane)
                // order, so which points share a wave (and, with pruning, its hit
                // window) is the same on every run.
                for (;;) {
                    float tt[C][NP];
                    int slot[C], rank[C];
                    uint64_t bal[C];
    #pragma unroll
                    for (int j = 0; j < C; ++j) {
                        if (pend[j]) {
    #pragma unroll
                            for (int a = 0; a < NP; ++a) tt[j][a] = __builtin_fmaf(alpha[j], p[j][a], th[j][a]);
                        }
                        bal[j] = __ballot(pend[j] && owner2);
                        rank[j] = __popcll(bal[j] & ((1ull << lane) - 1ull));
                    }
                    __syncthreads();  // the previous round is done with the list
                    if (lane == 0) {
    #pragma unroll
                        for (int j = 0; j < C; ++j) s_wcnt[j * kNW + wave] = __popcll(bal[j]);
                    }
                    __syncthreads();
                    int npend = 0, base[C];
    #pragma unroll
                    for (int j = 0; j < C; ++j) {
                        base[j] = 0;
                        for (int w = 0; w < kNW; ++w) {
                            if (w == wave) base[j] = npend;
                            npend += s_wcnt[j * kNW + w];
                        }
                    }
    #pragma unroll
                    for (int j = 0; j < C; ++j) {
                        slot[j] = pend[j] && owner2 ? base[j] + rank[j] : -1;
                        if (slot[j] >= 0) {
    #pragma unroll
                            for (int a = 0; a < NP; ++a) s_lth[slot[j]][a] = tt[j][a];
                        }
                    }
                    if constexpr (QS2 > 1) {
                        // the other lanes of a seed read its point
    #pragma unroll
                        for (int j = 0; j < C; ++j) slot[j] = __shfl(slot[j], slane2);
                    }
                    __syncthreads();
                    npend = __builtin_amdgcn_readfirstlane(npend);
                    if (npend == 0) break;
                    if (C == 1 && npend <= kWave) {
                        // npend points, parts = 256 / npend threads on each (the last
                        // 256 - parts * npend threads duplicate a part and are not read)
                        const int per = npend;
                        const int parts = kBlock / per;
                        const int used = parts * per;
                        const bool in = (int)threadIdx.x < used;
                        const int pt = in ? (int)threadIdx.x % per : 0, part = in ? (int)threadIdx.x / per : 0;
                        float lt[NP];
    #pragma unroll
                        for (int a = 0; a < NP; ++a) lt[a] = s_lth[pt][a];
                        s_red[threadIdx.x] = event_pass_split<D, PR>(d, s_hits, s_poff, ev, lt, nc, part, parts, in);
                        __syncthreads();  // every thread holds its point and partial
                        if ((int)threadIdx.x < per) {
                            float Rt = 0.0f;
                            for (int q = 0; q < parts; ++q) Rt += s_red[q * per + threadIdx.x];
                            s_lth[threadIdx.x][0] = Rt;
                        }
                        ls_pairs += (uint64_t)per * (uint64_t)ev.n;
                    } else {
                        const int per_round = kWave * C;
                        const int rounds = (npend + per_round - 1) / per_round;
                        for (int r = 0; r < rounds; ++r) {
                            Cands<C> cc;
                            bool live[C];
                            int ent[C];
    #pragma unroll
                            for (int j = 0; j < C; ++j) {
                                ent[j] = r * per_round + j * kWave + lane;
                                live[j] = ent[j] < npend;
                                float lt[NP];
    #pragma unroll
                                for (int a = 0; a < NP; ++a) lt[a] = live[j] ? s_lth[ent[j]][a] : 0.0f;
                                set_cand<D, C>(cc, j, lt);
                            }
                            __syncthreads();  // all waves hold the round's points before partials overwrite them
                            float racc[C][NA];
                            event_pass_part<D, C, PR>(d, s_hits, s_poff, ev, cc, nc, wave, kBlock / kWave, racc, live);
    #pragma unroll
                            for (int j = 0; j < C; ++j)
                                if (live[j]) s_lth[ent[j]][wave] = racc[j][0];
                        }
                        __syncthreads();
                        // ((wave 0 + wave 1) + wave 2) + wave 3, into slot 0
    #pragma unroll
                        for (int j = 0; j < C; ++j) {
                            const int e2 = (int)threadIdx.x + j * kBlock;
                            if (e2 < npend) {
                                const float* pr = s_lth[e2];
                                const float Rt = ((pr[0] + pr[1]) + pr[2]) + pr[3];
                                s_lth[e2][0] = Rt;
                            }
                        }
                        ls_pairs += (uint64_t)rounds * per_round * (uint64_t)ev.n;
                    }
                    __syncthreads();
    #pragma unroll
                    for (int j = 0; j < C; ++j) {
                        if (!pend[j]) continue;
                        ++nre[j];
                        const float Rt = s_lth[slot[j]][0];
                        if (Rt >= Rc[j] + d->armijo_c1 * alpha[j] * gp[j]) {
    #pragma unroll
                            for (int a = 0; a < NP; ++a) th[j][a] = tt[j][a];
                            if constexpr (U == 2) {
    #pragma unroll
                                for (int a = 0; a < NP; ++a) sq[j][a] = ds[a] * (alpha[j] * p[j][a]);
                            }
                            pend[j] = false;
                        } else if (++trial[j] >= d->ls_trials) {
                            pend[j] = false;
                            flags[j] |= RETINA_STALLED;
                        } else {
                            alpha[j] *= 0.5f;
                        }
                    }
                }
            }

            // FP64 Newton polish at sigma_final
            double T[C][NP];
    #pragma unroll
            for (int j = 0; j < C; ++j)
    #pragma unroll
                for (int a = 0; a < NP; ++a) T[j][a] = (double)th[j][a];
            const float sf = d->sigma_final;
            const float ncf = -kLog2e / (sf * sf);
            float Rfin[C];
            double step[C];
            bool pd[C];
            for (int it2 = 0; it2 < d->n_polish; ++it2) {
                // n_slope_steps counts on from the steps into the polish iterations
                const bool slope_pol = D == 2 && n_steps + it2 < d->n_slope_steps;
                Cands<C> ch, cl;
    #pragma unroll
                for (int j = 0; j < C; ++j) {
                    float hi[NP], lo[NP];
    #pragma unroll
                    for (int a = 0; a < NP; ++a) {
                        hi[a] = (float)T[j][a];
                        lo[a] = (float)(T[j][a] - (double)hi[a]);
                    }
                    set_cand<D, C>(ch, j, hi);
                    set_cand<D, C>(cl, j, lo);
                }
                float acc[C][NA];
                event_pass<D, C, true, true, PR, QS2>(d, s_hits, s_poff, ev, ch, cl, ncf, acc, wave_work, active);
    #pragma unroll
                for (int j = 0; j < C; ++j) {
                    double g[NP], H[NP][NP], A[NP][NP], dl[NP];
                    grad_hess<D, double>(acc[j], sf, g, H);
    #pragma unroll
                    for (int a = 0; a < NP; ++a)
    #pragma unroll
                        for (int b = 0; b < NP; ++b) A[a][b] = -H[a][b];
                    if (slope_pol) {
                        // offsets held: identity on the offset block and a zero offset
                        // gradient leave the Newton system of the slope block (its
                        // Cholesky factor is the block's own) and zero offset steps
    #pragma unroll
                        for (int a = 0; a < NP; ++a)
    #pragma unroll
                            for (int b = 0; b < 2; ++b) {
                                A[a][b] = a == b ? 1.0 : 0.0;
                                A[b][a] = a == b ? 1.0 : 0.0;
                            }
                        g[0] = 0.0;
                        g[1] = 0.0;
                    }
                    pd[j] = chol_solve<NP>(A, g, dl);
                    Rfin[j] = acc[j][0];
                    if (pd[j]) {
                        double s2 = 0.0;
    #pragma unroll
                        for (int a = 0; a < NP; ++a) {
                            T[j][a] += dl[a];
                            const double sd = (double)ds[a] * dl[a];
                            s2 += sd * sd;
                        }
                        step[j] = sqrt(s2);
                    } else {
                        step[j] = INFINITY;
                    }
                }
            }
    #pragma unroll
            for (int j = 0; j < C; ++j) {
                if (!pd[j]) flags[j] |= RETINA_NOT_PD;
                else if (step[j] <= (double)d->conv_tol * (double)sf) flags[j] |= RETINA_CONVERGED;
                if (!active[j] || !owner2) continue;
                const int sj = it.y + (wave * C + j) * SL2 + slane2;
                const int64_t gs = sbase + sj;
                double* o = d->s_theta + gs * 4;
    #pragma unroll
                for (int a = 0; a < 4; ++a) o[a] = a < NP ? T[j][a] : 0.0;
                d->s_R[gs] = Rfin[j];
                d->s_flags[gs] = flags[j];
                d->s_nreval[gs] = nre[j];
            }
            if (lane == 0 && wave_work) {
                const uint64_t per_pass = (uint64_t)ev.n * SL2;
                atomicAdd((unsigned long long*)&d->cnt->exec_pairs,
                          (unsigned long long)(per_pass * C * (uint64_t)(n_steps + d->n_polish)));
            }
            if (threadIdx.x == 0) {
                atomicAdd((unsigned long long*)&d->cnt->exec_pairs, (unsigned long long)ls_pairs);
                atomicAdd((unsigned long long*)&d->cnt->exec_rpairs, (unsigned long long)ls_pairs);
            }
            if (lane == 0 && wls_pairs) {
                atomicAdd((unsigned long long*)&d->cnt->exec_pairs, (unsigned long long)wls_pairs);
                atomicAdd((unsigned long long*)&d->cnt->exec_rpairs, (unsigned long long)wls_pairs);
            }
        };
        if constexpr (QS > 1) {
            const int r = min(ns - it.y, isz);
            if (r <= kNW * (kWave / kMaxSplitLanes)) item_body(std::integral_constant<int, kMaxSplitLanes>{});
            else if (r <= kNW * (kWave / (kMaxSplitLanes / 2))) item_body(std::integral_constant<int, kMaxSplitLanes / 2>{});
            else item_body(std::integral_constant<int, QS>{});
        } else {
            item_body(std::integral_constant<int, QS>{});
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- response
template <int D, int C, bool DERIV>
__global__ __launch_bounds__(kBlock) void k_response(const Desc* __restrict__ d, int tile_cap)
{
    constexpr int NP = 2 * D;
    constexpr int NA = Acc<D>::N;
    // dynamic LDS follows the static arrays: declared float4 so it starts 16-byte
    // aligned (the (x, y) hit pairs are read with 8-byte LDS loads)
    extern __shared__ float4 s_dyn[];
    float* s_hits = reinterpret_cast<float*>(s_dyn);
    __shared__ int s_poff[kMaxPlanes + 1];
    __shared__ int s_item;
    if (d->cnt->err) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // scalar: same in every lane
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t n_items = d->cnt->n_items;
    const float sig = d->resp_sigma;
    const float nc = -kLog2e / (sig * sig);
    const Cands<C> zero_c = {};
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&d->cnt->item, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= n_items) break;
        const int2 it0 = d->items[item];
        const int parts = d->resp_parts;
        const int part = it0.y % parts;
        const int2 it = make_int2(it0.x, (it0.y / parts) * d->seeds_per_item);  // (event, first theta)
        const int e = __builtin_amdgcn_readfirstlane(it.x);
        const EventView ev = begin_event(d, e, s_hits, s_poff, tile_cap, part, parts);
        const int64_t sbase = d->seed_off[e];
        const int ns = (int)(d->seed_off[e + 1] - sbase);
        Cands<C> c;
        bool active[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int sj = it.y + (wave * C + j) * kWave + lane;
            active[j] = sj < ns;
            float th[NP];
            if (d->resp_grid) {
                lattice_point<D>(d, active[j] ? sj : 0, th);
            } else {
                const float* src = d->in_theta + (sbase + (active[j] ? sj : 0)) * NP;
#pragma unroll
                for (int a = 0; a < NP; ++a) th[a] = active[j] ? src[a] : 0.0f;
            }
            set_cand<D, C>(c, j, th);
        }
        float acc[C][NA];
        event_pass<D, C, DERIV, false>(d, s_hits, s_poff, ev, c, zero_c, nc, acc);
        if (parts > 1) {
            // partial sums of this part of the hits; k_response_reduce adds the parts
#pragma unroll
            for (int j = 0; j < C; ++j) {
                if (!active[j]) continue;
                const int64_t gj = sbase + it.y + (wave * C + j) * kWave + lane;
                float* dst = d->resp_partial + ((int64_t)part * d->resp_ntheta + gj) * NA;
#pragma unroll
                for (int a = 0; a < NA; ++a) dst[a] = (DERIV || a == 0) ? acc[j][a] : 0.0f;
            }
            __syncthreads();
            continue;
        }
#pragma unroll
        for (int j = 0; j < C; ++j) {
            if (!active[j]) continue;
            const int64_t gj = sbase + it.y + (wave * C + j) * kWave + lane;
            d->out_R[gj] = acc[j][0];
            if (DERIV) {
                float g[NP], H[NP][NP];
                grad_hess<D, float>(acc[j], sig, g, H);
                if (d->want & RETINA_WANT_GRAD) {
#pragma unroll
                    for (int a = 0; a < NP; ++a) d->out_grad[gj * NP + a] = g[a];
                }
                if (d->want & RETINA_WANT_HESS) {
                    int q = 0;
#pragma unroll
                    for (int a = 0; a < NP; ++a)
#pragma unroll
                        for (int b = a; b < NP; ++b) d->out_hess[gj * (NP * (NP + 1) / 2) + q++] = H[a][b];
                }
            }
        }
        __syncthreads();
    }
}

// Sum of the parts' accumulators in part order, then the outputs as in k_response.
template <int D, bool DERIV>
__global__ __launch_bounds__(256) void k_response_reduce(const Desc* __restrict__ d, int64_t n_theta)
{
    constexpr int NP = 2 * D;
    constexpr int NA = Acc<D>::N;
    if (d->cnt->err) return;
    const float sig = d->resp_sigma;
    const int parts = d->resp_parts;
    for (int64_t gj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gj < n_theta;
         gj += (int64_t)gridDim.x * blockDim.x) {
        float acc[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) acc[a] = 0.0f;
        for (int q = 0; q < parts; ++q) {
            const float* src = d->resp_partial + ((int64_t)q * n_theta + gj) * NA;
#pragma unroll
            for (int a = 0; a < NA; ++a) acc[a] += src[a];
        }
        d->out_R[gj] = acc[0];
        if (DERIV) {
            float g[NP], H[NP][NP];
            grad_hess<D, float>(acc, sig, g, H);
            if (d->want & RETINA_WANT_GRAD) {
#pragma unroll
                for (int a = 0; a < NP; ++a) d->out_grad[gj * NP + a] = g[a];
            }
            if (d->want & RETINA_WANT_HESS) {
                int q = 0;
#pragma unroll
                for (int a = 0; a < NP; ++a)
#pragma unroll
                    for (int b = a; b < NP; ++b) d->out_hess[gj * (NP * (NP + 1) / 2) + q++] = H[a][b];
            }
        }
    }
}

void launch_response_reduce(const Desc* d, int D, bool deriv, int64_t n_theta, hipStream_t st)
{
    const dim3 g((unsigned)std::min<int64_t>((n_theta + 255) / 256, 4096)), b(256);
    if (D == 2) {
        if (deriv) hipLaunchKernelGGL((k_response_reduce<2, true>), g, b, 0, st, d, n_theta);
        else hipLaunchKernelGGL((k_response_reduce<2, false>), g, b, 0, st, d, n_theta);
    } else {
        if (deriv) hipLaunchKernelGGL((k_response_reduce<1, true>), g, b, 0, st, d, n_theta);
        else hipLaunchKernelGGL((k_response_reduce<1, false>), g, b, 0, st, d, n_theta);
    }
}

// ------------------------------------------------------------------ launch
int hot_seeds_per_item(const HotConfig& c) { return (kBlock / kWave) * kWave * c.cand / (c.split ? kSplitLanes : 1); }

size_t hot_lds_bytes(int meas_dim, const HotConfig& c)
{
    return (size_t)(c.tile_hits + (c.split ? kTilePadSplit : kTilePad)) * meas_dim * sizeof(float);
}

template <typename K>
static int occupancy(K kern, size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kBlock, lds) != hipSuccess) return 1;
    // LDS bound with the static and the dynamic part each rounded up to the
    // 512-byte allocation unit: the occupancy query has counted one work-group
    // more than fitted (a kernel 160 bytes under a third of the CU's LDS by the
    // plain sum, over it once the parts are rounded), and a persistent grid
    // sized by that count leaves the extra work-groups waiting for a slot
    hipFuncAttributes fa;
    int dev = 0, cu_lds = 0;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)) == hipSuccess && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
        cu_lds > 0) {
        auto up = [](size_t b) { return (b + 511) / 512 * 512; };
        const size_t per = up(fa.sharedSizeBytes) + up(lds);
        if (per > 0) nb = std::min<int>(nb, (int)((size_t)cu_lds / per));
    }
    return nb > 0 ? nb : 1;
}

int hot_max_blocks_per_cu(int D, const HotConfig& c, bool ascent)
{
    const size_t lds = hot_lds_bytes(D, c);
    if (ascent) {
        if (c.split) return D == 2 ? occupancy(k_ascent<2, 1, 0, false, kSplitLanes>, lds) : occupancy(k_ascent<1, 1, 0, false, kSplitLanes>, lds);
        if (D == 2) return c.cand == 2 ? occupancy(k_ascent<2, 2>, lds) : occupancy(k_ascent<2, 1>, lds);
        return c.cand == 2 ? occupancy(k_ascent<1, 2>, lds) : occupancy(k_ascent<1, 1>, lds);
    }
    if (D == 2) return c.cand == 2 ? occupancy(k_response<2, 2, true>, lds) : occupancy(k_response<2, 1, true>, lds);
    return c.cand == 2 ? occupancy(k_response<1, 2, true>, lds) : occupancy(k_response<1, 1, true>, lds);
}

void launch_ascent(const Desc* d, int D, const HotConfig& c, hipStream_t st)
{
    const size_t lds = hot_lds_bytes(D, c);
    const dim3 g(c.grid), b(kBlock);
    if (c.split && c.cand == 1 && c.update == 0) {
        // kSplitLanes lanes per seed (one candidate per lane, Newton steps)
        if (D == 2) {
            if (c.prune) hipLaunchKernelGGL((k_ascent<2, 1, 0, true, kSplitLanes>), g, b, lds, st, d, c.tile_hits);
            else hipLaunchKernelGGL((k_ascent<2, 1, 0, false, kSplitLanes>), g, b, lds, st, d, c.tile_hits);
        } else {
            if (c.prune) hipLaunchKernelGGL((k_ascent<1, 1, 0, true, kSplitLanes>), g, b, lds, st, d, c.tile_hits);
            else hipLaunchKernelGGL((k_ascent<1, 1, 0, false, kSplitLanes>), g, b, lds, st, d, c.tile_hits);
        }
        return;
    }
    if (c.prune) {
        // locality-pruned passes (truncated Newton)
        if (D == 2) {
            if (c.cand == 2) hipLaunchKernelGGL((k_ascent<2, 2, 0, true>), g, b, lds, st, d, c.tile_hits);
            else hipLaunchKernelGGL((k_ascent<2, 1, 0, true>), g, b, lds, st, d, c.tile_hits);
        } else {
            if (c.cand == 2) hipLaunchKernelGGL((k_ascent<1, 2, 0, true>), g, b, lds, st, d, c.tile_hits);
            else hipLaunchKernelGGL((k_ascent<1, 1, 0, true>), g, b, lds, st, d, c.tile_hits);
        }
        return;
    }
    if (c.update != 0) {
        // the alternative update rules run one candidate per lane
        if (D == 2) {
            if (c.update == 1) hipLaunchKernelGGL((k_ascent<2, 1, 1>), g, b, lds, st, d, c.tile_hits);
            else hipLaunchKernelGGL((k_ascent<2, 1, 2>), g, b, lds, st, d, c.tile_hits);
        } else {
            if (c.update == 1) hipLaunchKernelGGL((k_ascent<1, 1, 1>), g, b, lds, st, d, c.tile_hits);
            else hipLaunchKernelGGL((k_ascent<1, 1, 2>), g, b, lds, st, d, c.tile_hits);
        }
        return;
    }
    if (D == 2) {
        if (c.cand == 2) hipLaunchKernelGGL((k_ascent<2, 2>), g, b, lds, st, d, c.tile_hits);
        else hipLaunchKernelGGL((k_ascent<2, 1>), g, b, lds, st, d, c.tile_hits);
    } else {
        if (c.cand == 2) hipLaunchKernelGGL((k_ascent<1, 2>), g, b, lds, st, d, c.tile_hits);
        else hipLaunchKernelGGL((k_ascent<1, 1>), g, b, lds, st, d, c.tile_hits);
    }
}

void launch_response(const Desc* d, int D, const HotConfig& c, bool deriv, hipStream_t st)
{
    const size_t lds = hot_lds_bytes(D, c);
    const dim3 g(c.grid), b(kBlock);
#define RT_LAUNCH_RESP(DD, CC, DV) hipLaunchKernelGGL((k_response<DD, CC, DV>), g, b, lds, st, d, c.tile_hits)
    if (D == 2) {
        if (deriv) { if (c.cand == 2) RT_LAUNCH_RESP(2, 2, true); else RT_LAUNCH_RESP(2, 1, true); }
        else { if (c.cand == 2) RT_LAUNCH_RESP(2, 2, false); else RT_LAUNCH_RESP(2, 1, false); }
    } else {
        if (deriv) { if (c.cand == 2) RT_LAUNCH_RESP(1, 2, true); else RT_LAUNCH_RESP(1, 1, true); }
        else { if (c.cand == 2) RT_LAUNCH_RESP(1, 2, false); else RT_LAUNCH_RESP(1, 1, false); }
    }
#undef RT_LAUNCH_RESP
}

}  // namespace rt

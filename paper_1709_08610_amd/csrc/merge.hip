// Cluster the converged solutions of each event and keep the best of each
// cluster above R0 (Algorithm 1, last two steps).
//
// Per event (one work-group, persistent over events):
//   1. candidates = converged seeds with R >= R0, keyed (R desc, seed index
//      asc) and compacted;
//   2. bitonic sort of the keys (LDS when they fit, else a global scratch);
//   3. greedy leader clustering in key order, 256 candidates at a time:
//      every candidate first tests the leaders founded before its chunk (in
//      parallel; the first within d_merge wins, which is exactly what the
//      sequential rule gives since earlier leaders come first).  The chunk's
//      remaining candidates are resolved among themselves without walking
//      them in order: each gets the bit mask of its earlier remaining
//      neighbours within d_merge; in rounds, a candidate with a leader among
//      them becomes a member, one whose neighbours are all members (or none)
//      founds a leader.  The sequential rule gives the same split (a
//      candidate founds a leader exactly when no earlier leader lies within
//      d_merge), and a member joins its earliest leader neighbour, which is
//      the first leader founded among them.
// The cluster distance is the largest in-plane separation of the two lines
// over the detector's two end planes, in FP64.
#include "rt_internal.h"

namespace rt {

template <int D>
__device__ __forceinline__ double line_dist(const double* a, const double* b, double z0, double z1)
{
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double z = q == 0 ? z0 : z1;
        if (D == 2) {
            d = fmax(d, fabs((a[0] - b[0]) + (a[2] - b[2]) * z));
            d = fmax(d, fabs((a[1] - b[1]) + (a[3] - b[3]) * z));
        } else {
            d = fmax(d, fabs((a[0] - b[0]) + (a[1] - b[1]) * z));
        }
    }
    return d;
}

// KC / LC: candidates sorted in LDS and leaders cached in LDS (larger events
// use the global scratch for the rest); WPS: waves per SIMD the kernel must
// leave room for (the small-capacity shape runs several events per CU).
template <int D, int KC = kMergeKeyCap, int LC = kMergeLeaderCap, int WPS = 1>
__global__ __launch_bounds__(kBlock, WPS) void k_merge(const Desc* __restrict__ d)
{
    constexpr int NP = 2 * D;
    __shared__ uint64_t s_keys[KC];
    __shared__ double s_lth[LC][NP];
    __shared__ double s_cth[kBlock][NP];  // the chunk's candidate lines
    __shared__ int s_join[kBlock];
    __shared__ uint64_t s_lm[kBlock / kWave], s_um[kBlock / kWave];  // leader / unresolved masks of a chunk
    __shared__ int s_wcnt[kBlock / kWave];
    __shared__ int s_n;
    __shared__ int s_nl;
    __shared__ int s_flag;
    if (d->cnt->err) return;
    const int t = threadIdx.x;
    const int wave = t / kWave, lane = t & (kWave - 1);
    const double R0 = d->R0, dm = d->d_merge, z0 = d->z_first, z1 = d->z_last;
    for (int64_t e = blockIdx.x; e < d->n_events; e += gridDim.x) {
        const int64_t s0 = d->seed_off[e];
        const int ns = (int)(d->seed_off[e + 1] - s0);
        if (t == 0) { s_n = 0; s_nl = 0; s_flag = 0; }
        __syncthreads();
        // keys: LDS when they fit, else the event's slice of a 2x-seeds scratch (pow2 padding)
        uint64_t* keys = ns <= KC ? s_keys : d->m_keys + 2 * s0;
        int* lead = d->m_leader + s0;    // leader seed index (event-local)
        int* memb = d->m_members + s0;
        // 1. collect (order-preserving compaction)
        int evflag = 0;
        for (int j0 = 0; j0 < ns; j0 += kBlock) {
            const int j = j0 + t;
            bool take = false;
            uint64_t key = 0;
            if (j < ns) {
                const int f = d->s_flags[s0 + j];
                const float R = d->s_R[s0 + j];
                evflag |= f & RETINA_STALLED;
                take = (f & RETINA_CONVERGED) && (double)R >= R0;
                key = ((uint64_t)__float_as_uint(R) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)j);
            }
            const uint64_t m = __ballot(take);
            if (lane == 0) s_wcnt[wave] = __popcll(m);
            __syncthreads();
            int base = s_n;
            for (int w = 0; w < wave; ++w) base += s_wcnt[w];
            const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
            if (take) keys[base + __popcll(m & below)] = key;
            __syncthreads();
            if (t == 0) { int tot = 0; for (int w = 0; w < kBlock / kWave; ++w) tot += s_wcnt[w]; s_n += tot; }
            __syncthreads();
        }
        if (evflag) atomicOr(&s_flag, evflag);
        const int nc = s_n;
        // 2. sort descending (pad to a power of two with zero keys, which sort last)
        int np2 = 1;
        while (np2 < nc) np2 <<= 1;
        for (int i = nc + t; i < np2; i += kBlock) keys[i] = 0ull;
        __syncthreads();
        for (int k = 2; k <= np2; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int i = t; i < np2; i += kBlock) {
                    const int l = i ^ jj;
                    if (l > i) {
                        const uint64_t a = keys[i], b = keys[l];
                        const bool desc = (i & k) == 0;
                        if (desc ? (a < b) : (a > b)) { keys[i] = b; keys[l] = a; }
                    }
                }
                __syncthreads();
            }
        }
        // 3. greedy leader clustering
        for (int c0 = 0; c0 < nc; c0 += kBlock) {
            const int c = c0 + t;
            const int nl_old = s_nl;
            double th[NP];
            int sj = -1;
            if (c < nc) {
                sj = (int)(0xFFFFFFFFu - (uint32_t)(keys[c] & 0xFFFFFFFFull));
                const double* src = d->s_theta + (s0 + sj) * 4;
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    th[a] = src[a];
                    s_cth[t][a] = th[a];
                }
                int join = -1;
                for (int l = 0; l < nl_old; ++l) {
                    double lt[NP];
                    if (l < LC) {
#pragma unroll
                        for (int a = 0; a < NP; ++a) lt[a] = s_lth[l][a];
                    } else {
                        const double* ls = d->s_theta + (s0 + lead[l]) * 4;
#pragma unroll
                        for (int a = 0; a < NP; ++a) lt[a] = ls[a];
                    }
                    if (line_dist<D>(th, lt, z0, z1) <= dm) { join = l; break; }
                }
                s_join[t] = join;
            } else {
                s_join[t] = -2;
            }
            __syncthreads();
            // the chunk's unmatched candidates among themselves (see the top)
            constexpr int NW = kBlock / kWave;
            const bool un = c < nc && s_join[t] == -1;
            uint64_t nb[NW];  // earlier unmatched neighbours within d_merge, by chunk position
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                uint64_t m = 0;
                if (un) {
                    for (int k = 0; k < kWave; ++k) {
                        const int v = w * kWave + k;
                        if (v >= t) break;
                        if (s_join[v] != -1) continue;
                        double lt[NP];
#pragma unroll
                        for (int a = 0; a < NP; ++a) lt[a] = s_cth[v][a];
                        if (line_dist<D>(th, lt, z0, z1) <= dm) m |= 1ull << k;
                    }
                }
                nb[w] = m;
            }
            bool lead_u = false, done = !un;
            uint64_t m_un = __ballot(un);
            if (lane == 0) { s_lm[wave] = 0ull; s_um[wave] = m_un; }
            for (;;) {
                __syncthreads();
                bool any = false;
                uint64_t lm[NW], um[NW];
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    lm[w] = s_lm[w];
                    um[w] = s_um[w];
                    any = any || um[w] != 0ull;
                }
                if (!any) break;  // uniform: every thread read the same masks
                if (!done) {
                    bool hit_leader = false, open = false;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        hit_leader = hit_leader || (nb[w] & lm[w]) != 0ull;
                        open = open || (nb[w] & um[w]) != 0ull;
                    }
                    if (hit_leader) done = true;
                    else if (!open) { done = true; lead_u = true; }
                }
                const uint64_t ml = __ballot(lead_u), mu = __ballot(!done);
                __syncthreads();  // every thread has read the round's masks
                if (lane == 0) { s_lm[wave] = ml; s_um[wave] = mu; }
            }
            // indices: leaders in chunk order after the nl_old earlier ones; a
            // member joins its earliest leader neighbour
            {
                uint64_t lm[NW];
                int nl_new = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    lm[w] = s_lm[w];
                    nl_new += __popcll(lm[w]);
                }
                auto rank = [&](int v) {
                    int r = 0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        if (w < (v >> 6)) r += __popcll(lm[w]);
                        else if (w == (v >> 6)) r += __popcll(lm[w] & ((1ull << (v & 63)) - 1ull));
                    }
                    return nl_old + r;
                };
                if (un) {
                    if (lead_u) {
                        const int l = rank(t);
                        if (l < LC) {
#pragma unroll
                            for (int a = 0; a < NP; ++a) s_lth[l][a] = th[a];
                        }
                        lead[l] = sj;
                        memb[l] = 0;
                        s_join[t] = l;
                    } else {
                        int v = -1;
#pragma unroll
                        for (int w = NW - 1; w >= 0; --w) {
                            const uint64_t m = nb[w] & lm[w];
                            if (m) v = w * kWave + __builtin_ctzll(m);
                        }
                        s_join[t] = rank(v);
                    }
                }
                if (t == 0) s_nl = nl_old + nl_new;
            }
            __syncthreads();
            if (c < nc) atomicAdd(&memb[s_join[t]], 1);
            __syncthreads();
        }
        if (t == 0) {
            d->ev_ntracks[e] = s_nl;
            d->ev_flags[e] = s_flag;
        }
        __syncthreads();
    }
}

// Exclusive scan of per-event track counts into the caller's offsets, with
// the capacity check.  One work-group of 1024 threads.
__global__ __launch_bounds__(1024) void k_finalize(const Desc* __restrict__ d)
{
    __shared__ int64_t s_tmp[1024];
    if (d->cnt->err) return;
    const int t = threadIdx.x;
    const int64_t E = d->n_events;
    int64_t carry = 0;
    for (int64_t e0 = 0; e0 < E; e0 += 1024) {
        const int64_t e = e0 + t;
        const int64_t v = e < E ? d->ev_ntracks[e] : 0;
        s_tmp[t] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t add = t >= off ? s_tmp[t - off] : 0;
            __syncthreads();
            s_tmp[t] += add;
            __syncthreads();
        }
        const int64_t ex = s_tmp[t] - v;
        const int64_t tot = s_tmp[1023];
        __syncthreads();
        if (e < E) d->ev_toff[e] = carry + ex;
        carry += tot;
    }
    if (t == 0) {
        d->cnt->total_tracks = carry;
        d->ev_toff[E] = carry;
        // on overflow only the required total reaches the caller
        d->out_track_off[E] = carry;
        if (carry > d->out_capacity) atomicOr(&d->cnt->err, kErrCapacity);
    }
}

// Write tracks, event flags and optional per-seed results to the caller's
// arrays.  Grid-stride over events.
template <int D>
__global__ __launch_bounds__(kBlock) void k_emit(const Desc* __restrict__ d)
{
    constexpr int NP = 2 * D;
    if (d->cnt->err) return;
    for (int64_t e = blockIdx.x; e < d->n_events; e += gridDim.x) {
        const int64_t s0 = d->seed_off[e];
        const int64_t o = d->ev_toff[e];
        const int nl = d->ev_ntracks[e];
        if (threadIdx.x == 0) d->out_track_off[e] = o;
        for (int l = threadIdx.x; l < nl; l += blockDim.x) {
            const int sj = d->m_leader[s0 + l];
            const int64_t gs = s0 + sj;
            retina_track tr;
#pragma unroll
            for (int a = 0; a < 4; ++a) tr.theta[a] = a < NP ? d->s_theta[gs * 4 + a] : 0.0;
            tr.R = d->s_R[gs];
            tr.n_members = d->m_members[s0 + l];
            tr.seed_index = sj;
            tr.flags = d->s_flags[gs];
            d->out_tracks[o + l] = tr;
        }
        if (threadIdx.x == 0 && d->out_ev_flags) d->out_ev_flags[e] = d->ev_flags[e];
        const int ns = (int)(d->seed_off[e + 1] - s0);
        if (d->out_s_theta)
            for (int j = threadIdx.x; j < ns * NP; j += blockDim.x)
                d->out_s_theta[s0 * NP + j] = d->s_theta[(s0 + j / NP) * 4 + (j % NP)];
        if (d->out_s_R)
            for (int j = threadIdx.x; j < ns; j += blockDim.x) d->out_s_R[s0 + j] = d->s_R[s0 + j];
        if (d->out_s_flags)
            for (int j = threadIdx.x; j < ns; j += blockDim.x) d->out_s_flags[s0 + j] = d->s_flags[s0 + j];
        if (d->out_s_nreval)
            for (int j = threadIdx.x; j < ns; j += blockDim.x) d->out_s_nreval[s0 + j] = d->s_nreval[s0 + j];
    }
}

void launch_merge(const Desc* d, int D, int grid, bool small, hipStream_t st)
{
    // few seeds per event: small LDS caches and 4 work-groups per CU
    if (small) {
        if (D == 2) hipLaunchKernelGGL((k_merge<2, kMergeSmallKeys, kMergeSmallLeaders, 4>), dim3(grid * 4), dim3(kBlock), 0, st, d);
        else hipLaunchKernelGGL((k_merge<1, kMergeSmallKeys, kMergeSmallLeaders, 4>), dim3(grid * 4), dim3(kBlock), 0, st, d);
        return;
    }
    if (D == 2) hipLaunchKernelGGL(k_merge<2>, dim3(grid), dim3(kBlock), 0, st, d);
    else hipLaunchKernelGGL(k_merge<1>, dim3(grid), dim3(kBlock), 0, st, d);
}

void launch_finalize(const Desc* d, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, d);
}

void launch_emit(const Desc* d, int D, int grid, hipStream_t st)
{
    if (D == 2) hipLaunchKernelGGL(k_emit<2>, dim3(grid), dim3(kBlock), 0, st, d);
    else hipLaunchKernelGGL(k_emit<1>, dim3(grid), dim3(kBlock), 0, st, d);
}

}  // namespace rt

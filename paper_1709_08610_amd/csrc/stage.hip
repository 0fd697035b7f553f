// Hit staging and work planning.
//
// k_stage  validates each event's hits and counting-sorts them by plane
//          (stable: a hit keeps its input order within its plane), writing
//          per-(event, plane) offsets.  The hot kernels fold their sums per
//          plane, where z is constant, so the plane grouping is what lets the
//          per-hit work stay at six accumulators.
// k_plan   counts seeds per event, orders events longest first (hits x seeds)
//          and materialises the persistent kernels' (event, seed block)
//          work list.
#include "rt_internal.h"

namespace rt {

__global__ void k_reset(const Desc* __restrict__ d)
{
    // pruning: every event starts sortable; k_sort_planes clears the flag of an
    // event with a plane too long to sort
    if (d->ev_sorted)
        for (int64_t e = threadIdx.x; e < d->n_events; e += blockDim.x) d->ev_sorted[e] = 1;
    if (threadIdx.x == 0) {
        Counters* c = d->cnt;
        c->item = 0;
        c->err = 0;
        c->n_items = 0;
        c->total_tracks = 0;
        c->total_seeds = 0;
        c->exec_pairs = 0;
        c->exec_rpairs = 0;
    }
    if (threadIdx.x < kXcds) d->cnt->xq_cursor[threadIdx.x][0] = 0;
    if (threadIdx.x <= kXcds) d->cnt->xq_start[threadIdx.x] = 0;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int lane = threadIdx.x & (kWave - 1);
    return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

// One wavefront per event.  Pass 1: histogram of planes (LDS atomics) and
// validation.  Exclusive scan over planes.  Pass 2: stable scatter, ranks
// from wave ballots per distinct plane in the chunk.
constexpr int kPlaneBits = 6;  // plane numbers < RETINA_MAX_PLANES = 64
static_assert(kMaxPlanes <= (1 << kPlaneBits) && kMaxPlanes <= kWave, "one lane per plane, 6-bit plane numbers");

__global__ __launch_bounds__(kBlock) void k_stage(const Desc* __restrict__ d)
{
    constexpr int NW = kBlock / kWave;
    __shared__ int s_cnt[NW][kMaxPlanes];  // per wave: plane counts, then a chunk's counts
    __shared__ int s_bad;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // scalar: same in every lane
    const int lane = threadIdx.x & (kWave - 1);
    const int P = d->n_planes;
    const int D = d->meas_dim;
    const int64_t E = d->n_events;
    int* cnt = s_cnt[wave];
    uint32_t err = 0;
    // one event per work-group; wave w validates, counts and scatters the w-th
    // quarter of its hits (contiguous, whole 64-hit chunks), so the placement
    // is the one-wave stable counting sort's
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int64_t a = d->in_off[e];
        const int64_t b = d->in_off[e + 1];
        if ((e == 0 && a != 0) || b < a || b > d->n_hits) {
            err |= kErrOffsets;
            continue;  // uniform over the work-group
        }
        __syncthreads();  // the previous event is done with s_cnt and s_bad
        if (threadIdx.x == 0) s_bad = 0;
        if (lane < P) cnt[lane] = 0;
        const int64_t q = ((b - a + NW - 1) / NW + kWave - 1) / kWave * kWave;
        const int64_t wa = min(b, a + wave * q), wb = min(b, wa + q);
        __syncthreads();
        bool bad = false;
        for (int64_t k0 = wa; k0 < wb; k0 += kWave) {
            const int64_t k = k0 + lane;
            if (k < wb) {
                const int p = d->in_plane[k];
                const float x = d->in_x[k];
                const float y = D == 2 ? d->in_y[k] : 0.0f;
                if (p < 0 || p >= P) { err |= kErrPlane; bad = true; }
                else atomicAdd(&cnt[p], 1);
                if (!isfinite(x) || !isfinite(y)) { err |= kErrCoord; bad = true; }
            }
        }
        if (__any(bad) && lane == 0) s_bad = 1;
        __syncthreads();
        if (s_bad) continue;  // uniform: read after the barrier
        // lane p: the event's hits of planes < p (an exclusive scan of the
        // totals) plus those of plane p in the waves before this one
        int tot = 0, before = 0;
        if (lane < P) {
            for (int w = 0; w < NW; ++w) {
                const int c = s_cnt[w][lane];
                tot += c;
                if (w < wave) before += c;
            }
        }
        int incl = tot;
        for (int off = 1; off < kWave; off <<= 1) {
            const int v = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += v;
        }
        int cursor = (int)a + incl - tot + before;  // lane p: this wave's next free slot of plane p
        if (wave == 0) {
            int32_t* po = d->plane_off + e * (P + 1);
            if (lane < P) po[lane] = (int)a + incl - tot;
            if (lane == 0) {
                po[P] = (int)b;
                d->ev_nhits[e] = (int)(b - a);
            }
        }
        __syncthreads();  // every wave has read the counts before its row is reused
        // per 64-hit chunk: the lanes holding the same plane are those whose
        // plane numbers agree bit by bit (one ballot per bit), a hit's slot is
        // its plane's cursor plus the number of earlier lanes of that plane
        // (stable), and the last lane of each plane hands the chunk's count
        // to the lane that keeps the plane's cursor
        const uint64_t gt = lane == kWave - 1 ? 0ull : (~0ull << (lane + 1));
        for (int64_t k0 = wa; k0 < wb; k0 += kWave) {
            const int64_t k = k0 + lane;
            const bool live = k < wb;
            const int p = live ? d->in_plane[k] : 0;
            float2 v = make_float2(0.0f, 0.0f);
            if (live) {
                v.x = d->in_x[k];
                if (D == 2) v.y = d->in_y[k];
            }
            uint64_t same = __ballot(live);
#pragma unroll
            for (int bit = 0; bit < kPlaneBits; ++bit) {
                const bool on = live && ((p >> bit) & 1);
                const uint64_t m = __ballot(on);
                same &= on ? m : ~m;
            }
            const int base = __shfl(cursor, p, kWave);
            const int pos = base + __popcll(same & lanemask_lt());
            if (lane < P) cnt[lane] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (live && (same & gt) == 0) cnt[p] = __popcll(same);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane < P) cursor += cnt[lane];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (live) {
                if (D == 2) reinterpret_cast<float2*>(d->hits)[pos] = v;
                else d->hits[pos] = v.x;
            }
        }
    }
    if (err) atomicOr(&d->cnt->err, err);
}

// ---------------------------------------------------------------- sorting
// Pruned passes need every plane segment of an event sorted by x (the first
// measured coordinate).  One work-group per (event, plane) segment of at most
// kSortCap hits: a bitonic sort in LDS, padding with +inf keys; an event with
// a longer segment is marked unsorted and its passes stay unpruned.
constexpr int kSortCap = 4096;

__global__ __launch_bounds__(kBlock) void k_sort_planes(const Desc* __restrict__ d)
{
    __shared__ float2 s_h[kSortCap];
    if (d->cnt->err) return;
    const int P = d->n_planes;
    const int D = d->meas_dim;
    const int64_t n_seg = d->n_events * P;
    for (int64_t sg = blockIdx.x; sg < n_seg; sg += gridDim.x) {
        const int64_t e = sg / P;
        const int p = (int)(sg % P);
        const int32_t* po = d->plane_off + e * (P + 1);
        const int lo = po[p], len = po[p + 1] - po[p];
        if (len > kSortCap) {
            if (threadIdx.x == 0) d->ev_sorted[e] = 0;
            continue;
        }
        if (len <= 1) continue;
        int n_pad = 1;
        while (n_pad < len) n_pad <<= 1;
        for (int i = threadIdx.x; i < n_pad; i += blockDim.x) {
            float2 v = make_float2(INFINITY, 0.0f);
            if (i < len) {
                if (D == 2) v = reinterpret_cast<const float2*>(d->hits)[lo + i];
                else v.x = d->hits[lo + i];
            }
            s_h[i] = v;
        }
        __syncthreads();
        for (int k = 2; k <= n_pad; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < n_pad; i += blockDim.x) {
                    const int l = i ^ j;
                    if (l > i) {
                        const float2 a = s_h[i], b = s_h[l];
                        const bool up = (i & k) == 0;
                        if (up ? (a.x > b.x) : (a.x < b.x)) { s_h[i] = b; s_h[l] = a; }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < len; i += blockDim.x) {
            if (D == 2) reinterpret_cast<float2*>(d->hits)[lo + i] = s_h[i];
            else d->hits[lo + i] = s_h[i].x;
        }
        __syncthreads();  // the LDS buffer is reused by the next segment
    }
}

// ---------------------------------------------------------------- planning
// Work list for the persistent kernels.  seed_mode 0: lattice (same count per
// event); 1: explicit seeds (in_seed_off); 2: response thetas (in_theta_off);
// 3: response on the lattice (grid search; same count per event).
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* s_tmp, int64_t& total)
{
    // blockDim.x == 1024
    const int t = threadIdx.x;
    s_tmp[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t add = t >= off ? s_tmp[t - off] : 0;
        __syncthreads();
        s_tmp[t] += add;
        __syncthreads();
    }
    const int64_t incl = s_tmp[t];
    total = s_tmp[1023];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(1024) void k_plan(const Desc* __restrict__ d, int mode)
{
    __shared__ int64_t s_tmp[1024];
    __shared__ uint64_t s_key[kPlanSortCap];
    const int t = threadIdx.x;
    const int64_t E = d->n_events;
    if (d->cnt->err) return;
    if (mode < 0) mode = d->seed_mode;
    const int64_t* so = mode == 1 ? d->in_seed_off : (mode == 2 ? d->in_theta_off : nullptr);
    const int64_t lat = (int64_t)d->lattice_n[0] * d->lattice_n[1];
    uint32_t err = 0;
    if (so && t == 0 && so[0] != 0) err |= (mode == 1 ? kErrSeedOff : kErrThetaOff);
    // global seed offsets in event order
    int64_t carry = 0;
    for (int64_t e0 = 0; e0 < E; e0 += 1024) {
        const int64_t e = e0 + t;
        int64_t n = 0;
        if (e < E) {
            n = so ? so[e + 1] - so[e] : lat;
            if (n < 0) { err |= (mode == 1 ? kErrSeedOff : kErrThetaOff); n = 0; }
        }
        int64_t tot;
        const int64_t ex = block_excl_scan(n, s_tmp, tot);
        if (e < E) d->seed_off[e] = carry + ex;
        carry += tot;
    }
    if (t == 0) { d->seed_off[E] = carry; d->cnt->total_seeds = carry; }
    if (err) atomicOr(&d->cnt->err, err);
    __syncthreads();
    if (d->cnt->err) return;
    // longest first: key = cost (hits x seeds) high, event index low (ties: batch order)
    const bool sorted = E <= kPlanSortCap;
    int64_t n_pad = 1;
    while (n_pad < E) n_pad <<= 1;
    if (sorted) {
        for (int64_t e = t; e < n_pad; e += 1024) {
            uint64_t key = 0;
            if (e < E) {
                const uint64_t ns = (uint64_t)(d->seed_off[e + 1] - d->seed_off[e]);
                uint64_t cost = (uint64_t)d->ev_nhits[e] * ns + ns;  // + ns: hit-less events still cost
                if (cost > 0xFFFFFFFFull) cost = 0xFFFFFFFFull;
                key = (cost << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)e);
            }
            s_key[e] = key;
        }
        __syncthreads();
        for (int64_t k = 2; k <= n_pad; k <<= 1) {
            for (int64_t j = k >> 1; j > 0; j >>= 1) {
                for (int64_t i = t; i < n_pad; i += 1024) {
                    const int64_t l = i ^ j;
                    if (l > i) {
                        const uint64_t a = s_key[i], b = s_key[l];
                        const bool desc = (i & k) == 0;
                        if (desc ? (a < b) : (a > b)) { s_key[i] = b; s_key[l] = a; }
                    }
                }
                __syncthreads();
            }
        }
        for (int64_t r = t; r < E; r += 1024) d->order[r] = (int32_t)(0xFFFFFFFFu - (uint32_t)(s_key[r] & 0xFFFFFFFFull));
    } else {
        for (int64_t r = t; r < E; r += 1024) d->order[r] = (int32_t)r;
    }
    __syncthreads();
    const int spi = d->seeds_per_item;
    if (mode == 0 || mode == 1) {
        // track finding: the events of rank r (longest first) go to XCD queue
        // r % kXcds.  Each queue holds first the full items of its events, then
        // their part-filled last items (cheaper, so the work ends on short
        // items), both in rank order; with half_parts an event's part-filled
        // seeds form one or two half items (the split shape runs a half item
        // with 8 or 16 lanes per seed on all four waves).  Full and part-filled
        // item counts are summed together, packed into the low and high halves
        // of one word.
        __shared__ int64_t s_qcarry[kXcds], s_qstart[kXcds + 1], s_qfull[kXcds];
        for (int pass = 0; pass < 2; ++pass) {
            if (t < kXcds) s_qcarry[t] = 0;
            __syncthreads();
            for (int64_t r0 = 0; r0 < E; r0 += 1024) {
                const int64_t r = r0 + t;  // r % kXcds == t % kXcds (1024 is a multiple of kXcds)
                int64_t nf = 0, np = 0;
                int e = 0;
                if (r < E) {
                    e = d->order[r];
                    const int64_t ns = d->seed_off[e + 1] - d->seed_off[e];
                    nf = ns / spi;
                    const int64_t rem = ns % spi;
                    np = rem == 0 ? 0 : (d->half_parts && 2 * rem > spi ? 2 : 1);
                }
                const int64_t v = nf | (np << 32);
                // inclusive prefix over this chunk's ranks of the same queue
                s_tmp[t] = v;
                __syncthreads();
                for (int off = kXcds; off < 1024; off <<= 1) {
                    const int64_t add = t >= off ? s_tmp[t - off] : 0;
                    __syncthreads();
                    s_tmp[t] += add;
                    __syncthreads();
                }
                const int q = t % kXcds;
                const int64_t ex = s_tmp[t] - v + s_qcarry[q];
                if (pass == 1 && r < E) {
                    const int64_t exf = ex & 0xFFFFFFFFll, exp_ = ex >> 32;
                    for (int64_t b = 0; b < nf; ++b) {
                        const int64_t it = s_qstart[q] + exf + b;
                        if (it < d->items_cap) d->items[it] = make_int2(e, (int)b);
                    }
                    for (int64_t k = 0; k < np; ++k) {
                        const int64_t it = s_qstart[q] + s_qfull[q] + exp_ + k;
                        const int blk = d->half_parts ? ~(int)(2 * nf + k) : (int)nf;
                        if (it < d->items_cap) d->items[it] = make_int2(e, blk);
                    }
                }
                __syncthreads();
                if (t < kXcds) s_qcarry[t] += s_tmp[1024 - kXcds + t];  // the chunk's last rank of queue t
                __syncthreads();
            }
            if (pass == 0 && t == 0) {
                int64_t acc = 0;
                for (int q = 0; q < kXcds; ++q) {
                    s_qstart[q] = acc;
                    s_qfull[q] = s_qcarry[q] & 0xFFFFFFFFll;
                    acc += s_qfull[q] + (s_qcarry[q] >> 32);
                }
                s_qstart[kXcds] = acc;
            }
            __syncthreads();
        }
        if (t <= kXcds) d->cnt->xq_start[t] = s_qstart[t];
        if (t == 0) {
            if (s_qstart[kXcds] > d->items_cap) atomicOr(&d->cnt->err, kErrSeedOff);
            d->cnt->n_items = s_qstart[kXcds];
        }
        return;
    }
    // items in rank order
    const int parts = (mode == 2 || mode == 3) && d->resp_parts > 1 ? d->resp_parts : 1;
    carry = 0;
    for (int64_t r0 = 0; r0 < E; r0 += 1024) {
        const int64_t r = r0 + t;
        int64_t nb = 0;
        int e = 0;
        if (r < E) {
            e = d->order[r];
            const int64_t ns = d->seed_off[e + 1] - d->seed_off[e];
            nb = (ns + spi - 1) / spi * parts;
        }
        int64_t tot;
        const int64_t ex = block_excl_scan(nb, s_tmp, tot);
        if (r < E) {
            for (int64_t b = 0; b < nb; ++b) {
                const int64_t it = carry + ex + b;
                if (it < d->items_cap) d->items[it] = make_int2(e, (int)b);
            }
        }
        carry += tot;
    }
    if (t == 0) {
        if (carry > d->items_cap) atomicOr(&d->cnt->err, kErrSeedOff);
        d->cnt->n_items = carry;
    }
}

void launch_reset(const Desc* d, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, d);
}

void launch_stage(const Desc* d, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_stage, dim3(grid), dim3(kBlock), 0, st, d);
}

void launch_sort_planes(const Desc* d, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_sort_planes, dim3(grid), dim3(kBlock), 0, st, d);
}

void launch_plan_tracks(const Desc* d, hipStream_t st)
{
    // the host sets seed_mode 0 (lattice) or 1 (explicit) in the descriptor; the
    // kernel's mode argument mirrors it so a captured graph needs no host branch
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, d, -1);
}

void launch_plan_response(const Desc* d, hipStream_t st)
{
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, d, 2);
}

void launch_plan_grid(const Desc* d, hipStream_t st)
{
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, d, 3);
}

}  // namespace rt

// Grid-search Artificial Retina (Section 2: the steps of the grid-based AR
// algorithms that the optimisation method replaces).  The response at every
// cell comes from k_response on lattice candidates; this file finds the
// groups of cells with a high response and estimates one track per group:
//   peak      a cell whose response reaches R0 and exceeds that of each of its
//             (up to 8) neighbours inside the grid; an equal neighbour means
//             no peak
//   estimate  the response-weighted mean of the cell centres of the peak's
//             3 x 3 neighbourhood (cells inside the grid), in FP64
// Three passes over chunks of kGridChunk consecutive cells of one event:
// count the peaks of every chunk, scan the counts (first track slot of each
// chunk and event), then write the tracks in cell order.
#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kGridThreads = 256;
constexpr int kGridRound = 4 * kGridThreads;  // cells per round: 4 consecutive per thread
static_assert(kGridChunk % kGridRound == 0, "a chunk is whole rounds");

__device__ __forceinline__ bool grid_peak(const float* __restrict__ G, int n0, int n1, int i0, int i1, float R0)
{
    const float r = G[(int64_t)i0 * n1 + i1];
    if (!(r >= R0)) return false;
    for (int a = -1; a <= 1; ++a) {
        const int j0 = i0 + a;
        if (j0 < 0 || j0 >= n0) continue;
        for (int b = -1; b <= 1; ++b) {
            const int j1 = i1 + b;
            if ((a == 0 && b == 0) || j1 < 0 || j1 >= n1) continue;
            if (!(r > G[(int64_t)j0 * n1 + j1])) return false;
        }
    }
    return true;
}

// peak flags of this thread's 4 consecutive cells of a round (bit k: cell k)
__device__ __forceinline__ uint32_t round_flags(const Desc* __restrict__ d, const float* __restrict__ G,
                                                int64_t n_cells, int64_t c0)
{
    const int n0 = d->lattice_n[0], n1 = d->lattice_n[1];
    uint32_t f = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t c = c0 + k;
        if (c < n_cells && grid_peak(G, n0, n1, (int)(c / n1), (int)(c % n1), d->grid_R0)) f |= 1u << k;
    }
    return f;
}

// exclusive prefix over the work-group (kGridThreads threads) and the total
__device__ __forceinline__ uint32_t block_excl(uint32_t v, uint32_t* s, uint32_t& total)
{
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < kGridThreads; off <<= 1) {
        const uint32_t add = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    const uint32_t incl = s[t];
    total = s[kGridThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kGridThreads) void k_grid_count(const Desc* __restrict__ d)
{
    __shared__ uint32_t s_tmp[kGridThreads];
    if (d->cnt->err) return;
    const int nch = d->grid_chunks;
    const int64_t e = blockIdx.x / nch, ch = blockIdx.x % nch;
    const int64_t n_cells = (int64_t)d->lattice_n[0] * d->lattice_n[1];
    const float* G = d->out_R + e * n_cells;
    uint32_t cnt = 0;
    for (int r = 0; r < kGridChunk / kGridRound; ++r) {
        const int64_t c0 = ch * kGridChunk + (int64_t)r * kGridRound + 4 * threadIdx.x;
        cnt += __popc(round_flags(d, G, n_cells, c0));
    }
    uint32_t total;
    block_excl(cnt, s_tmp, total);
    if (threadIdx.x == 0) d->grid_cnt[blockIdx.x] = (int32_t)total;
}

// one work-group: exclusive scan of the chunk counts in (event, chunk) order
__global__ __launch_bounds__(1024) void k_grid_scan(const Desc* __restrict__ d, int64_t n_total)
{
    __shared__ int64_t s_tmp[1024];
    if (d->cnt->err) return;
    const int t = threadIdx.x;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < n_total; b0 += 1024) {
        const int64_t b = b0 + t;
        const int64_t v = b < n_total ? d->grid_cnt[b] : 0;
        s_tmp[t] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t add = t >= off ? s_tmp[t - off] : 0;
            __syncthreads();
            s_tmp[t] += add;
            __syncthreads();
        }
        if (b < n_total) d->grid_base[b] = carry + s_tmp[t] - v;
        carry += s_tmp[1023];
        __syncthreads();
    }
    if (t == 0) {
        d->cnt->total_tracks = carry;
        d->out_track_off[d->n_events] = carry;  // on overflow only the required total reaches the caller
        if (carry > d->out_capacity) atomicOr(&d->cnt->err, kErrCapacity);
    }
}

template <int D>
__global__ __launch_bounds__(kGridThreads) void k_grid_emit(const Desc* __restrict__ d)
{
    __shared__ uint32_t s_tmp[kGridThreads];
    if (d->cnt->err) return;
    const int nch = d->grid_chunks;
    const int64_t e = blockIdx.x / nch, ch = blockIdx.x % nch;
    const int n0 = d->lattice_n[0], n1 = d->lattice_n[1];
    const int64_t n_cells = (int64_t)n0 * n1;
    const float* G = d->out_R + e * n_cells;
    const float R0 = d->grid_R0;
    int64_t slot = d->grid_base[blockIdx.x];
    if (ch == 0 && threadIdx.x == 0) d->out_track_off[e] = slot;
    for (int r = 0; r < kGridChunk / kGridRound; ++r) {
        const int64_t c0 = ch * kGridChunk + (int64_t)r * kGridRound + 4 * threadIdx.x;
        const uint32_t f = round_flags(d, G, n_cells, c0);
        uint32_t total;
        uint32_t rank = block_excl(__popc(f), s_tmp, total);
        for (int k = 0; k < 4; ++k) {
            if (!(f >> k & 1u)) continue;
            const int64_t c = c0 + k;
            const int i0 = (int)(c / n1), i1 = (int)(c % n1);
            double w = 0.0, m0 = 0.0, m1 = 0.0;
            int members = 0;
            for (int a = -1; a <= 1; ++a) {
                const int j0 = i0 + a;
                if (j0 < 0 || j0 >= n0) continue;
                const double v0 = d->lat_coord[j0];
                for (int b = -1; b <= 1; ++b) {
                    const int j1 = i1 + b;
                    if (j1 < 0 || j1 >= n1) continue;
                    const float g = G[(int64_t)j0 * n1 + j1];
                    const double v1 = d->lat_coord[n0 + j1];
                    w += (double)g;
                    m0 += (double)g * v0;
                    m1 += (double)g * v1;
                    members += g >= R0;
                }
            }
            double t0 = d->lat_coord[i0];
            double t1 = d->lat_coord[n0 + i1];
            if (w > 0.0) { t0 = m0 / w; t1 = m1 / w; }
            retina_track tr;
            if constexpr (D == 2) { tr.theta[0] = 0.0; tr.theta[1] = 0.0; tr.theta[2] = t0; tr.theta[3] = t1; }
            else { tr.theta[0] = t1; tr.theta[1] = t0; tr.theta[2] = 0.0; tr.theta[3] = 0.0; }
            tr.R = G[c];
            tr.n_members = members;
            tr.seed_index = (int32_t)c;
            tr.flags = 0;
            d->out_tracks[slot + rank] = tr;
            ++rank;
        }
        slot += total;
    }
}

}  // namespace

void launch_grid_peaks(const Desc* d, int meas_dim, int64_t n_chunks_total, hipStream_t st)
{
    if (n_chunks_total <= 0) return;
    const dim3 g((unsigned)n_chunks_total), b(kGridThreads);
    hipLaunchKernelGGL(k_grid_count, g, b, 0, st, d);
    hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(1024), 0, st, d, n_chunks_total);
    if (meas_dim == 2) hipLaunchKernelGGL(k_grid_emit<2>, g, b, 0, st, d);
    else hipLaunchKernelGGL(k_grid_emit<1>, g, b, 0, st, d);
}

}  // namespace rt

// Internal layout shared by libretina's translation units (host and device).
// Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/retina.h"

namespace rt {

constexpr int kMaxPlanes = RETINA_MAX_PLANES;
constexpr int kMaxSigma = RETINA_MAX_SIGMA;
constexpr int kBlock = 256;          // threads per work-group of the hot kernels
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kMergeKeyCap = 8192;   // candidates sorted in LDS by the merge kernel
constexpr int kMergeLeaderCap = 1024;// leader parameters cached in LDS by the merge kernel
constexpr int kMergeSmallKeys = 1024;   // the same for sparse seeding (several events per CU)
constexpr int kMergeSmallLeaders = 256;
constexpr int kPlanSortCap = 8192;   // events ordered longest-first in LDS (larger: batch order)

// error bits raised by device-side validation
enum : uint32_t {
    kErrOffsets = 1u,     // event offsets decreasing / not starting at 0
    kErrCoord = 2u,       // non-finite hit coordinate
    kErrPlane = 4u,       // plane index out of range
    kErrSeedOff = 8u,     // explicit seed offsets invalid
    kErrSeedVal = 16u,    // non-finite explicit seed
    kErrThetaOff = 32u,   // response theta offsets invalid
    kErrThetaVal = 64u,   // non-finite response theta
    kErrCapacity = 128u   // tracks do not fit the caller's array
};

// Largest side of a seed lattice or search grid: the cell-centre coordinates
// of both dimensions travel in the descriptor (Desc::lat_coord).
constexpr int kMaxLatticeSide = RETINA_MAX_LATTICE_SIDE;

// Work-groups of a launch are dealt to the XCDs round-robin by index; the
// ascent keeps one work queue per XCD so that an event's work items share the
// XCD's L2 (the event's hits are then read from HBM once).
constexpr int kXcds = 8;

// device-side counters (one cache line each to avoid false sharing of atomics)
struct Counters {
    uint32_t item;          // persistent work queue cursor
    uint32_t pad0[15];
    uint32_t err;           // validation error bits
    uint32_t pad1[15];
    int64_t n_items;        // produced by the planner
    int64_t total_tracks;   // produced by the finaliser
    int64_t total_seeds;
    uint64_t exec_pairs;    // hit-candidate pairs the hot kernel executed (all lanes)
    uint64_t exec_rpairs;   // ... of which in R-only line-search passes
    int64_t pad2[3];
    uint32_t xq_cursor[kXcds][16];  // per-XCD queue cursors of the ascent (one line each)
    int64_t xq_start[kXcds + 1];    // queue x holds items [xq_start[x], xq_start[x + 1])
};

// Everything a launch needs; lives in device memory and is refreshed by one
// host-to-device copy per call, so captured graphs stay valid across batches.
struct Desc {
    // geometry
    int32_t meas_dim, n_planes;
    float plane_z[kMaxPlanes];
    float z_first, z_last;       // detector end planes (merge distance)
    float z_ref;                 // RMS plane position (Newton-CG scaling)
    // caller inputs
    int32_t mem_pad;
    int64_t n_events;
    int64_t n_hits;
    const int64_t* in_off;
    const float* in_x;
    const float* in_y;
    const int32_t* in_plane;
    // staged hits (sorted by plane inside each event)
    float* hits;                 // meas_dim 2: (x, y) pairs; meas_dim 1: x
    int32_t* plane_off;          // n_events * (n_planes + 1), global hit offsets
    int32_t* ev_nhits;           // n_events
    // seeds
    int32_t seed_mode;
    int32_t lattice_n[2];
    float lattice_lo[2], lattice_hi[2];
    const double* in_seeds;
    const int64_t* in_seed_off;
    int64_t* seed_off;           // n_events + 1 (global seed offsets, event order)
    // response inputs
    const float* in_theta;
    const int64_t* in_theta_off; // NULL: single event
    uint32_t want;
    float resp_sigma;
    int32_t resp_parts;          // hit parts per (event, theta block): 1, or a split for few items
    int64_t resp_ntheta;
    float* resp_partial;         // resp_parts x n_theta x accumulators (parts > 1)
    float* out_R;
    float* out_grad;
    float* out_hess;
    // grid search: k_response takes its candidates from the lattice fields
    int32_t resp_grid;
    float grid_R0;
    int32_t grid_chunks;         // peak-pass chunks per event
    int32_t* grid_cnt;           // n_events * grid_chunks peak counts
    int64_t* grid_base;          // n_events * grid_chunks first track slot of each chunk
    // method parameters
    int32_t n_sigma;
    float sigma[kMaxSigma];
    float sigma_final;
    int32_t n_final_steps, n_polish, ls_trials, n_slope_steps;
    float armijo_c1, step_cap, small_step, conv_tol, R0, d_merge;
    float prune_u;               // > 0: skip hits farther than sqrt(prune_u) sigma in x from every candidate
    int32_t* ev_sorted;          // n_events: 1 when every plane segment is sorted by x (pruning allowed)
    // work items
    int32_t seeds_per_item;
    int32_t half_parts;          // 1: an event's part-filled seeds go in items of seeds_per_item / 2
    int32_t* order;              // events, longest first
    // (event, block * parts + part): seeds [block * seeds_per_item, ...); with
    // half_parts a negative block ~b is half-block b: [b * seeds_per_item / 2, ...)
    int2* items;
    int64_t items_cap;
    // per-seed results (pool)
    double* s_theta;             // n_seeds * 4
    float* s_R;
    int32_t* s_flags;
    int32_t* s_nreval;
    // merge results (pool, indexed like seeds)
    int32_t* m_leader;           // leader seed index within event
    int32_t* m_members;
    uint64_t* m_keys;            // 2 * n_seeds: sort scratch of events too large for LDS
    int32_t* ev_ntracks;         // n_events
    int32_t* ev_flags;           // n_events
    int64_t* ev_toff;            // n_events + 1: track offsets before the capacity check
    // caller outputs
    retina_track* out_tracks;
    int64_t out_capacity;
    int64_t* out_track_off;      // n_events + 1
    int32_t* out_ev_flags;
    double* out_s_theta;
    float* out_s_R;
    int32_t* out_s_flags;
    int32_t* out_s_nreval;
    // device counters
    Counters* cnt;
    // theta offsets {0, n_theta} of a one-event response call without caller
    // offsets (in_theta_off then points here, inside the device copy)
    int64_t single_off[2];
    // Cell-centre coordinates of the seed lattice / search grid, formed on the
    // host: dimension 0 in [0, lattice_n[0]), dimension 1 in [lattice_n[0],
    // lattice_n[0] + lattice_n[1]); each the FP32 rounding of
    // lo + (i + 1/2)(hi - lo)/n formed in FP64.  Only the used entries are
    // uploaded; must stay the last member.
    float lat_coord[2 * kMaxLatticeSide];
};

// launchers (one per translation unit); all asynchronous on `st`
void launch_reset(const Desc* d, hipStream_t st);
void launch_stage(const Desc* d, int grid, hipStream_t st);
void launch_sort_planes(const Desc* d, int grid, hipStream_t st);
void launch_plan_tracks(const Desc* d, hipStream_t st);
void launch_plan_response(const Desc* d, hipStream_t st);
void launch_plan_grid(const Desc* d, hipStream_t st);

struct HotConfig {
    int cand;        // candidates per lane (1, 2)
    int tile_hits;   // LDS capacity in hits
    int grid;        // persistent work-groups
    int update = 0;  // ascent update rule: 0 Newton, 1 gradient, 2 BFGS (cand 1)
    int prune = 0;   // locality-pruned passes (hits sorted by x per plane first)
    int staged = 0;  // hits already staged by the caller's previous launch (learned seeding)
    int split = 0;   // ascent: several lanes per seed (cand 1, Newton), smaller work items
    int small_merge = 0;  // merge with small LDS caches, several events per CU
};
int hot_seeds_per_item(const HotConfig& c);
void launch_ascent(const Desc* d, int meas_dim, const HotConfig& c, hipStream_t st);
void launch_response(const Desc* d, int meas_dim, const HotConfig& c, bool deriv, hipStream_t st);
void launch_response_reduce(const Desc* d, int meas_dim, bool deriv, int64_t n_theta, hipStream_t st);
size_t hot_lds_bytes(int meas_dim, const HotConfig& c);
int hot_max_blocks_per_cu(int meas_dim, const HotConfig& c, bool ascent);

void launch_merge(const Desc* d, int meas_dim, int grid, bool small, hipStream_t st);
void launch_finalize(const Desc* d, hipStream_t st);
void launch_emit(const Desc* d, int meas_dim, int grid, hipStream_t st);

constexpr int kGridChunk = 8192;     // cells per work-group of the peak passes
void launch_grid_peaks(const Desc* d, int meas_dim, int64_t n_chunks_total, hipStream_t st);

}  // namespace rt

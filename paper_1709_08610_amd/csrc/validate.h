// Host-side argument checks of the C-ABI entry points.  Plain C++ on the
// caller's arguments (no device calls, no allocation), so the same code runs
// inside libretina and in a CPU build under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Each check returns RETINA_OK or an error code
// with its message in `Check::msg`.
#pragma once
#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/retina.h"

namespace rtv {

struct Check {
    int code = RETINA_OK;
    char msg[256] = {0};
};

inline int bad(Check& k, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
inline int bad(Check& k, int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(k.msg, sizeof(k.msg), fmt, ap);
    va_end(ap);
    k.code = code;
    return code;
}

// meas_dim, plane count and finite plane positions
inline int geometry(Check& k, const retina_geometry* g)
{
    if (!g) return bad(k, RETINA_ERR_INVALID_ARG, "geometry is NULL");
    if (g->meas_dim != 1 && g->meas_dim != 2)
        return bad(k, RETINA_ERR_INVALID_ARG, "meas_dim must be 1 or 2 (got %d)", g->meas_dim);
    if (g->n_planes < 1 || g->n_planes > RETINA_MAX_PLANES)
        return bad(k, RETINA_ERR_INVALID_ARG, "n_planes must be in [1, %d] (got %d)", RETINA_MAX_PLANES,
                   g->n_planes);
    if (!g->plane_z) return bad(k, RETINA_ERR_INVALID_ARG, "plane_z is NULL");
    for (int p = 0; p < g->n_planes; ++p)
        if (!isfinite(g->plane_z[p])) return bad(k, RETINA_ERR_INVALID_ARG, "plane_z[%d] is not finite", p);
    return RETINA_OK;
}

// the hit batch descriptor (array contents are checked on the device)
inline int hits(Check& k, const retina_geometry* g, const retina_hits* h)
{
    if (!h) return bad(k, RETINA_ERR_INVALID_ARG, "hits is NULL");
    if (h->mem != RETINA_MEM_HOST && h->mem != RETINA_MEM_DEVICE)
        return bad(k, RETINA_ERR_INVALID_ARG, "hits.mem must be RETINA_MEM_HOST or RETINA_MEM_DEVICE");
    if (h->n_events < 0) return bad(k, RETINA_ERR_INVALID_ARG, "n_events < 0");
    if (h->n_events > 0x7FFFFFFF) return bad(k, RETINA_ERR_INVALID_ARG, "n_events too large");
    if (!h->event_offsets) return bad(k, RETINA_ERR_INVALID_ARG, "event_offsets is NULL");
    if (h->n_events > 0 && (!h->x || !h->plane))
        return bad(k, RETINA_ERR_INVALID_ARG, "hit arrays x / plane are NULL");
    if (h->n_events > 0 && g->meas_dim == 2 && !h->y)
        return bad(k, RETINA_ERR_INVALID_ARG, "hit array y is NULL with meas_dim 2");
    return RETINA_OK;
}

// n + 1 host offsets: off[0] = 0, non-decreasing
inline bool offsets_ok(const int64_t* off, int64_t n)
{
    if (off[0] != 0) return false;
    for (int64_t i = 0; i < n; ++i)
        if (off[i + 1] < off[i]) return false;
    return true;
}

// cell counts of a seed lattice or search grid
inline int lattice_sides(Check& k, const int32_t* n)
{
    for (int i = 0; i < 2; ++i)
        if (n[i] < 1 || n[i] > RETINA_MAX_LATTICE_SIDE)
            return bad(k, RETINA_ERR_INVALID_ARG, "lattice / grid side %d must be in [1, %d]", n[i],
                       RETINA_MAX_LATTICE_SIDE);
    return RETINA_OK;
}

// retina_response's scalar arguments and output pointers
inline int response_args(Check& k, const retina_hits* h, const float* theta, int64_t n_theta,
                         const int64_t* theta_offsets, float sigma, uint32_t want, const float* R,
                         const float* grad, const float* hess)
{
    if (!(sigma > 0.0f) || !isfinite(sigma)) return bad(k, RETINA_ERR_INVALID_ARG, "sigma must be finite and > 0");
    if (n_theta < 0) return bad(k, RETINA_ERR_INVALID_ARG, "n_theta < 0");
    if (want & ~(uint32_t)(RETINA_WANT_R | RETINA_WANT_GRAD | RETINA_WANT_HESS))
        return bad(k, RETINA_ERR_INVALID_ARG, "unknown want bits 0x%x", want);
    if (!theta_offsets && h->n_events != 1)
        return bad(k, RETINA_ERR_INVALID_ARG, "theta_offsets may be NULL only with one event");
    if (n_theta > 0 && (!theta || !R)) return bad(k, RETINA_ERR_INVALID_ARG, "theta / R is NULL");
    if (n_theta > 0 && (want & RETINA_WANT_GRAD) && !grad) return bad(k, RETINA_ERR_INVALID_ARG, "grad is NULL");
    if (n_theta > 0 && (want & RETINA_WANT_HESS) && !hess) return bad(k, RETINA_ERR_INVALID_ARG, "hess is NULL");
    return RETINA_OK;
}

// retina_find_tracks' method constants, seeding and output arguments
inline int method_params(Check& k, const retina_params* P, int64_t capacity, const retina_track* tracks,
                         const int64_t* track_offsets)
{
    if (!P) return bad(k, RETINA_ERR_INVALID_ARG, "params is NULL");
    if (P->n_sigma < 0 || P->n_sigma > RETINA_MAX_SIGMA)
        return bad(k, RETINA_ERR_INVALID_ARG, "n_sigma must be in [0, %d]", RETINA_MAX_SIGMA);
    if (P->n_sigma > 0 && !P->sigma) return bad(k, RETINA_ERR_INVALID_ARG, "sigma is NULL");
    for (int i = 0; i < P->n_sigma; ++i)
        if (!(P->sigma[i] > 0.0f) || !isfinite(P->sigma[i]))
            return bad(k, RETINA_ERR_INVALID_ARG, "sigma[%d] must be finite and > 0", i);
    if (!(P->sigma_final > 0.0f) || !isfinite(P->sigma_final))
        return bad(k, RETINA_ERR_INVALID_ARG, "sigma_final must be finite and > 0");
    if (P->n_final_steps < 0 || P->n_polish < 1 || P->ls_trials < 1 || P->n_slope_steps < 0)
        return bad(k, RETINA_ERR_INVALID_ARG, "step counts: n_final_steps >= 0, n_polish >= 1, ls_trials >= 1");
    if (P->n_sigma + P->n_final_steps > 64 || P->n_polish > 16 || P->ls_trials > 16)
        return bad(k, RETINA_ERR_INVALID_ARG, "step counts too large");
    const float fp[] = {P->armijo_c1, P->step_cap_sigmas, P->small_step_sigmas, P->conv_tol, P->R0, P->d_merge};
    for (float v : fp)
        if (!isfinite(v)) return bad(k, RETINA_ERR_INVALID_ARG, "method constants must be finite");
    if (!(P->step_cap_sigmas > 0.0f) || !(P->d_merge >= 0.0f) || !(P->conv_tol > 0.0f))
        return bad(k, RETINA_ERR_INVALID_ARG, "step_cap_sigmas, conv_tol must be > 0 and d_merge >= 0");
    if (P->seed_mode != RETINA_SEED_LATTICE && P->seed_mode != RETINA_SEED_EXPLICIT)
        return bad(k, RETINA_ERR_INVALID_ARG, "unknown seed_mode %d", P->seed_mode);
    if (P->update != RETINA_UPDATE_NEWTON && P->update != RETINA_UPDATE_GRADIENT && P->update != RETINA_UPDATE_BFGS)
        return bad(k, RETINA_ERR_INVALID_ARG, "unknown update rule %d", P->update);
    if (!isfinite(P->prune_u) || P->prune_u < 0.0f)
        return bad(k, RETINA_ERR_INVALID_ARG, "prune_u must be finite and >= 0");
    if (P->prune_u > 0.0f && P->update != RETINA_UPDATE_NEWTON)
        return bad(k, RETINA_ERR_INVALID_ARG, "pruned passes run with the truncated-Newton rule only");
    if (P->seed_mode == RETINA_SEED_LATTICE) {
        if (P->lattice_n[0] < 1 || P->lattice_n[1] < 1 || P->lattice_n[0] > RETINA_MAX_LATTICE_SIDE ||
            P->lattice_n[1] > RETINA_MAX_LATTICE_SIDE || (int64_t)P->lattice_n[0] * P->lattice_n[1] > (1 << 24))
            return bad(k, RETINA_ERR_INVALID_ARG, "lattice_n must be in [1, %d] with at most 2^24 seeds",
                       RETINA_MAX_LATTICE_SIDE);
        for (int i = 0; i < 2; ++i)
            if (!isfinite(P->lattice_lo[i]) || !isfinite(P->lattice_hi[i]))
                return bad(k, RETINA_ERR_INVALID_ARG, "lattice box must be finite");
    } else if (!P->seeds || !P->seed_offsets) {
        return bad(k, RETINA_ERR_INVALID_ARG, "explicit seeds / seed_offsets are NULL");
    }
    if (capacity < 0) return bad(k, RETINA_ERR_INVALID_ARG, "capacity < 0");
    if (!track_offsets) return bad(k, RETINA_ERR_INVALID_ARG, "track_offsets is NULL");
    if (capacity > 0 && !tracks) return bad(k, RETINA_ERR_INVALID_ARG, "tracks is NULL");
    return RETINA_OK;
}

// host explicit seeds: every value finite and within the FP32 range (the
// ascent's precision); checked in FP64, since converting a value beyond the
// FP32 range is undefined in C++
inline int host_seeds(Check& k, const double* seeds, int64_t n_values)
{
    for (int64_t i = 0; i < n_values; ++i)
        if (!(fabs(seeds[i]) <= (double)FLT_MAX))
            return bad(k, RETINA_ERR_INVALID_ARG, "an explicit seed is NaN or infinite in FP32");
    return RETINA_OK;
}

// Bump allocation of 256-byte aligned pieces from a fixed workspace of `cap`
// bytes; `used` advances only on success.
inline int arena_take(Check& k, size_t cap, size_t& used, size_t bytes, size_t* offset)
{
    const size_t want = ((bytes < 16 ? 16 : bytes) + 255) & ~(size_t)255;
    if (want < bytes || used > cap || want > cap - used)
        return bad(k, RETINA_ERR_CAPACITY,
                   "the call needs more than the %zu bytes of the fixed device workspace "
                   "(%zu in use, %zu more requested)",
                   cap, used, want);
    *offset = used;
    used += want;
    return RETINA_OK;
}

}  // namespace rtv

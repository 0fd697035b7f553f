// CPU driver for libretina's host-side argument checks (csrc/validate.h),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py.  Every case states the status it expects; the
// program exits non-zero on the first mismatch.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../paper_1709_08610_amd/csrc/validate.h"

static int failures = 0;

static void expect(const char* what, int got, int want, const rtv::Check& k)
{
    if (got != want) {
        fprintf(stderr, "FAIL %s: got %d want %d (%s)\n", what, got, want, k.msg);
        ++failures;
    }
}

#define CASE(what, call, want)       \
    do {                             \
        rtv::Check k_;               \
        int r_ = (call);             \
        expect(what, r_, want, k_);  \
    } while (0)

int main()
{
    const int OK = RETINA_OK, BAD = RETINA_ERR_INVALID_ARG, CAP = RETINA_ERR_CAPACITY;
    std::vector<float> z(26);
    for (int p = 0; p < 26; ++p) z[p] = 20.0f + 730.0f * p / 25.0f;
    retina_geometry g = {2, 26, z.data()};

    // geometry
    CASE("geometry ok", rtv::geometry(k_, &g), OK);
    CASE("geometry null", rtv::geometry(k_, nullptr), BAD);
    {
        retina_geometry b = g;
        b.meas_dim = 3;
        CASE("meas_dim 3", rtv::geometry(k_, &b), BAD);
        b = g;
        b.n_planes = RETINA_MAX_PLANES + 1;
        CASE("too many planes", rtv::geometry(k_, &b), BAD);
        b.n_planes = 0;
        CASE("no planes", rtv::geometry(k_, &b), BAD);
        b = g;
        b.plane_z = nullptr;
        CASE("plane_z null", rtv::geometry(k_, &b), BAD);
        std::vector<float> zn = z;
        zn[25] = NAN;
        b = g;
        b.plane_z = zn.data();
        CASE("plane_z nan", rtv::geometry(k_, &b), BAD);
        zn[25] = INFINITY;
        CASE("plane_z inf", rtv::geometry(k_, &b), BAD);
    }

    // hits
    std::vector<int64_t> off = {0, 3, 3, 7};
    std::vector<float> x(7, 1.0f), y(7, 2.0f);
    std::vector<int32_t> pl(7, 0);
    retina_hits h = {RETINA_MEM_HOST, 3, off.data(), x.data(), y.data(), pl.data()};
    CASE("hits ok", rtv::hits(k_, &g, &h), OK);
    CASE("hits null", rtv::hits(k_, &g, nullptr), BAD);
    {
        retina_hits b = h;
        b.mem = 7;
        CASE("hits mem", rtv::hits(k_, &g, &b), BAD);
        b = h;
        b.n_events = -1;
        CASE("negative events", rtv::hits(k_, &g, &b), BAD);
        b = h;
        b.n_events = (int64_t)1 << 40;
        CASE("too many events", rtv::hits(k_, &g, &b), BAD);
        b = h;
        b.y = nullptr;
        CASE("y null, meas_dim 2", rtv::hits(k_, &g, &b), BAD);
        retina_geometry g1 = g;
        g1.meas_dim = 1;
        CASE("y null, meas_dim 1", rtv::hits(k_, &g1, &b), OK);
        b = h;
        b.n_events = 0;
        b.x = nullptr;
        b.plane = nullptr;
        b.y = nullptr;
        CASE("empty batch, no arrays", rtv::hits(k_, &g, &b), OK);
    }

    // offsets
    CASE("offsets ok", rtv::offsets_ok(off.data(), 3) ? OK : BAD, OK);
    {
        std::vector<int64_t> o2 = {1, 3};
        CASE("offsets start", rtv::offsets_ok(o2.data(), 1) ? OK : BAD, BAD);
        std::vector<int64_t> o3 = {0, 5, 4, 9};
        CASE("offsets decrease", rtv::offsets_ok(o3.data(), 3) ? OK : BAD, BAD);
        std::vector<int64_t> o4 = {0};
        CASE("offsets zero events", rtv::offsets_ok(o4.data(), 0) ? OK : BAD, OK);
    }

    // lattice sides
    {
        int32_t n1[2] = {64, 64}, n2[2] = {0, 64}, n3[2] = {64, RETINA_MAX_LATTICE_SIDE + 1};
        CASE("lattice ok", rtv::lattice_sides(k_, n1), OK);
        CASE("lattice zero", rtv::lattice_sides(k_, n2), BAD);
        CASE("lattice too big", rtv::lattice_sides(k_, n3), BAD);
    }

    // response arguments
    {
        std::vector<float> th(16), R(4), G(16), H(40);
        std::vector<int64_t> to = {0, 2, 2, 4};
        const uint32_t all = RETINA_WANT_R | RETINA_WANT_GRAD | RETINA_WANT_HESS;
        CASE("response ok", rtv::response_args(k_, &h, th.data(), 4, to.data(), 0.03f, all, R.data(), G.data(), H.data()), OK);
        CASE("sigma 0", rtv::response_args(k_, &h, th.data(), 4, to.data(), 0.0f, all, R.data(), G.data(), H.data()), BAD);
        CASE("sigma nan", rtv::response_args(k_, &h, th.data(), 4, to.data(), NAN, all, R.data(), G.data(), H.data()), BAD);
        CASE("sigma inf", rtv::response_args(k_, &h, th.data(), 4, to.data(), INFINITY, all, R.data(), G.data(), H.data()), BAD);
        CASE("n_theta < 0", rtv::response_args(k_, &h, th.data(), -1, to.data(), 0.03f, all, R.data(), G.data(), H.data()), BAD);
        CASE("want bits", rtv::response_args(k_, &h, th.data(), 4, to.data(), 0.03f, 8u, R.data(), G.data(), H.data()), BAD);
        CASE("offsets null, 3 events", rtv::response_args(k_, &h, th.data(), 4, nullptr, 0.03f, all, R.data(), G.data(), H.data()), BAD);
        CASE("grad null", rtv::response_args(k_, &h, th.data(), 4, to.data(), 0.03f, all, R.data(), nullptr, H.data()), BAD);
        CASE("hess null", rtv::response_args(k_, &h, th.data(), 4, to.data(), 0.03f, all, R.data(), G.data(), nullptr), BAD);
        CASE("R only, no grad/hess", rtv::response_args(k_, &h, th.data(), 4, to.data(), 0.03f, RETINA_WANT_R, R.data(), nullptr, nullptr), OK);
        CASE("no thetas, null arrays", rtv::response_args(k_, &h, nullptr, 0, to.data(), 0.03f, all, nullptr, nullptr, nullptr), OK);
    }

    // method parameters
    {
        float sig[7] = {4, 2, 1, 0.5f, 0.25f, 0.125f, 0.0625f};
        retina_params P;
        memset(&P, 0, sizeof(P));
        P.n_sigma = 7;
        P.sigma = sig;
        P.sigma_final = 0.03f;
        P.n_final_steps = 3;
        P.n_polish = 2;
        P.ls_trials = 4;
        P.armijo_c1 = 0.25f;
        P.step_cap_sigmas = 2.0f;
        P.small_step_sigmas = 0.5f;
        P.conv_tol = 1e-3f;
        P.R0 = 8.0f;
        P.d_merge = 0.03f;
        P.seed_mode = RETINA_SEED_LATTICE;
        P.lattice_n[0] = P.lattice_n[1] = 64;
        P.lattice_lo[0] = P.lattice_lo[1] = -0.3f;
        P.lattice_hi[0] = P.lattice_hi[1] = 0.3f;
        std::vector<retina_track> tr(8);
        std::vector<int64_t> toff(4);
        CASE("params ok", rtv::method_params(k_, &P, 8, tr.data(), toff.data()), OK);
        CASE("params null", rtv::method_params(k_, nullptr, 8, tr.data(), toff.data()), BAD);
        retina_params Q = P;
        Q.n_sigma = RETINA_MAX_SIGMA + 1;
        CASE("n_sigma", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        float bad_sig[7] = {4, 2, -1, 0.5f, 0.25f, 0.125f, 0.0625f};
        Q.sigma = bad_sig;
        CASE("negative sigma", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.sigma_final = NAN;
        CASE("sigma_final nan", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.n_polish = 0;
        CASE("no polish", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.ls_trials = 17;
        CASE("ls_trials", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.armijo_c1 = INFINITY;
        CASE("armijo inf", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.d_merge = -1.0f;
        CASE("d_merge < 0", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.seed_mode = 5;
        CASE("seed_mode", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.update = 9;
        CASE("update rule", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.prune_u = 30.0f;
        Q.update = RETINA_UPDATE_BFGS;
        CASE("prune with BFGS", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.lattice_n[0] = 8192;
        Q.lattice_n[1] = 8192;
        CASE("lattice > 2^24 seeds", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.lattice_hi[1] = NAN;
        CASE("lattice box nan", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        Q = P;
        Q.seed_mode = RETINA_SEED_EXPLICIT;
        CASE("explicit without seeds", rtv::method_params(k_, &Q, 8, tr.data(), toff.data()), BAD);
        CASE("capacity < 0", rtv::method_params(k_, &P, -1, tr.data(), toff.data()), BAD);
        CASE("track_offsets null", rtv::method_params(k_, &P, 8, tr.data(), nullptr), BAD);
        CASE("tracks null", rtv::method_params(k_, &P, 8, nullptr, toff.data()), BAD);
        CASE("capacity 0, tracks null", rtv::method_params(k_, &P, 0, nullptr, toff.data()), OK);
    }

    // explicit host seeds (rounded to FP32)
    {
        std::vector<double> s = {0.0, 0.1, 0.2, 0.3, 1e39, 0.0, 0.0, 0.0};
        CASE("seeds ok", rtv::host_seeds(k_, s.data(), 4), OK);
        s[3] = -3.0e38;
        CASE("seed near the FP32 limit", rtv::host_seeds(k_, s.data(), 4), OK);
        CASE("seed overflows FP32", rtv::host_seeds(k_, s.data(), 8), BAD);
        s[4] = NAN;
        CASE("seed nan", rtv::host_seeds(k_, s.data(), 8), BAD);
        CASE("no seeds", rtv::host_seeds(k_, nullptr, 0), OK);
    }

    // fixed-workspace bump allocation
    {
        const size_t cap = 1 << 20;
        size_t used = 0, o1 = 1, o2 = 1, o3 = 1;
        CASE("take 1", rtv::arena_take(k_, cap, used, 100, &o1), OK);
        CASE("take 2", rtv::arena_take(k_, cap, used, 4096, &o2), OK);
        if (o1 != 0 || o2 != 256 || used != 256 + 4096) {
            fprintf(stderr, "FAIL arena layout %zu %zu %zu\n", o1, o2, used);
            ++failures;
        }
        CASE("take too much", rtv::arena_take(k_, cap, used, cap, &o3), CAP);
        if (used != 256 + 4096 || o3 != 1) {
            fprintf(stderr, "FAIL arena moved on a refusal\n");
            ++failures;
        }
        CASE("take SIZE_MAX", rtv::arena_take(k_, cap, used, SIZE_MAX, &o3), CAP);
        CASE("take the rest", rtv::arena_take(k_, cap, used, cap - used, &o3), OK);
        CASE("take past the end", rtv::arena_take(k_, cap, used, 1, &o3), CAP);
    }

    if (failures) {
        fprintf(stderr, "%d host-check case(s) failed\n", failures);
        return 1;
    }
    printf("host checks: all cases passed\n");
    return 0;
}

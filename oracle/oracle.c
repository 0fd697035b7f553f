/*
 * FP64 CPU oracle for the optimisation-based Artificial Retina
 * (Borisyak, Ustyuzhanin, Derkach, Belous, "Numerical optimization for
 * Artificial Retina Algorithm", arXiv:1709.08610).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * Everything is plain FP64 with direct loops: no blocking, no per-plane
 * factoring, no fusion.  Inputs arrive as the generator's FP32 values and are
 * widened exactly.
 *
 * Contents (each function names the passage it follows):
 *   oracle_response        Eq. (1) with the in-plane distance, plus its
 *                          gradient and Hessian (Section 2, Section 3)
 *   oracle_newton_cg       the truncated-Newton direction (Section 3, TN;
 *                          Nocedal & Wright line-search Newton-CG)
 *   oracle_ascend          one multi-start trajectory: sigma continuation,
 *                          Newton-CG, backtracking Armijo line search, FP64
 *                          Newton polish (Algorithm 1, inner loops)
 *   oracle_merge           cluster the converged solutions and keep the
 *                          highest response per cluster above R0
 *                          (Algorithm 1, last two steps)
 *   oracle_find_tracks     Algorithm 1 end to end over a batch of events
 *   oracle_bfgs_update     the quasi-Newton update of the BFGS rule
 *   oracle_polish          Newton polish of arbitrary points (used by the
 *                          brute-force grid cross-check)
 *   oracle_grid_search     the grid-search Artificial Retina the method is
 *                          compared with (Section 2, its four usual steps)
 *
 * Parameter layout: meas_dim D = 2 gives theta = (x0, y0, tx, ty); D = 1
 * gives theta = (x0, tx).  n_par = 2*D.  Hessians are returned packed upper
 * triangular, row-major: (00,01,..,0n, 11,12,.., nn).
 *
 * Parity status: every function here is pinned by the CPU tests (closed
 * forms, finite differences, least-squares fixed points, brute-force grids,
 * invariances); see the test files for which pin covers which function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXP 4
#define CG_RTOL 1e-4  /* relative CG forcing term */

/* Method parameters; mirrors the Python-side ctypes Structure in
 * oracle/__init__.py.  Single precision where the method's inputs are FP32
 * values (both sides consume the same FP32 numbers). */
typedef struct {
    int32_t n_sigma;          /* continuation stages */
    const float* sigma;       /* [n_sigma] */
    float sigma_final;
    int32_t n_final_steps;    /* steps at sigma_final after the stages */
    int32_t n_polish;         /* FP64 Newton polish iterations at sigma_final */
    int32_t ls_trials;        /* step lengths 1, 1/2, 1/4, ... */
    float armijo_c1;
    float step_cap_sigmas;    /* cap on the scaled step, in units of sigma */
    float small_step_sigmas;  /* scaled Newton steps at or below this (in sigma) skip the line search */
    int32_t n_slope_steps;    /* D = 2: the first n_slope_steps steps, counted on into the
                                 polish iterations, move (tx, ty) only */
    float conv_tol;           /* converged iff |D delta| <= conv_tol*sigma_final on the last polish */
    float R0;                 /* response threshold */
    float d_merge;            /* cluster radius (end-plane distance) */
    int32_t lattice_n[2];
    float lattice_lo[2];
    float lattice_hi[2];
    int32_t update;           /* 0 truncated Newton, 1 normalised gradient, 2 BFGS */
} oracle_params;

enum { OR_CONVERGED = 1, OR_STALLED = 2, OR_NOT_PD = 4, OR_NEGCURV = 8 };

/* ------------------------------------------------------------------------- */
/* Eq. (1): R(theta) = sum_k exp(-s(x_k, theta)^2 / sigma^2), with s the
 * Euclidean distance between the hit and the track's intersection with the
 * hit's plane (Section 3; for D = 1 the distance within the plane, Fig. 1).
 * With residuals r = x - x0 - tx*z (and r_y likewise), v = dr/dtheta^T * r:
 *   grad R = (2/sigma^2) sum_k e_k v_k
 *   Hess R = sum_k e_k [ (4/sigma^4) v_k v_k^T - (2/sigma^2) Phi_k ]
 * where Phi_k = sum over measured coordinates of phi phi^T, phi = (1, z) in
 * that coordinate's (x0, tx) slots.                                          */
static void response_one(int D, const double* pz, int64_t n, const double* x, const double* y,
                         const int32_t* pl, const double* th, double sigma,
                         double* R, double* g, double* H /* full n_par x n_par */)
{
    const int np = 2 * D;
    const double s2 = sigma * sigma;
    double r_acc = 0.0, g_acc[MAXP] = {0}, h_acc[MAXP][MAXP] = {{0}};
    for (int64_t k = 0; k < n; ++k) {
        const double z = pz[pl[k]];
        double v[MAXP] = {0}, phi[2][MAXP] = {{0}};
        double d2;
        if (D == 2) {
            const double rx = x[k] - th[0] - th[2] * z;
            const double ry = y[k] - th[1] - th[3] * z;
            d2 = rx * rx + ry * ry;
            /* phi_x = (1,0,z,0), phi_y = (0,1,0,z) */
            phi[0][0] = 1.0; phi[0][2] = z;
            phi[1][1] = 1.0; phi[1][3] = z;
            for (int a = 0; a < np; ++a) v[a] = rx * phi[0][a] + ry * phi[1][a];
        } else {
            const double r = x[k] - th[0] - th[1] * z;
            d2 = r * r;
            phi[0][0] = 1.0; phi[0][1] = z;
            for (int a = 0; a < np; ++a) v[a] = r * phi[0][a];
        }
        const double e = exp(-d2 / s2);
        r_acc += e;
        for (int a = 0; a < np; ++a) g_acc[a] += (2.0 / s2) * e * v[a];
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
                double phiphi = 0.0;
                for (int c = 0; c < D; ++c) phiphi += phi[c][a] * phi[c][b];
                h_acc[a][b] += e * ((4.0 / (s2 * s2)) * v[a] * v[b] - (2.0 / s2) * phiphi);
            }
    }
    *R = r_acc;
    if (g) for (int a = 0; a < np; ++a) g[a] = g_acc[a];
    if (H) for (int a = 0; a < np; ++a) for (int b = 0; b < np; ++b) H[a * np + b] = h_acc[a][b];
}

static double response_only(int D, const double* pz, int64_t n, const double* x, const double* y,
                            const int32_t* pl, const double* th, double sigma)
{
    double R;
    response_one(D, pz, n, x, y, pl, th, sigma, &R, NULL, NULL);
    return R;
}

/* Widen an event's FP32 inputs to FP64. Caller frees *xd (one block). */
static void widen(int D, int64_t n, const float* x, const float* y, double** xd, double** yd)
{
    double* blk = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)D);
    for (int64_t k = 0; k < n; ++k) blk[k] = (double)x[k];
    if (D == 2) for (int64_t k = 0; k < n; ++k) blk[n + k] = (double)y[k];
    *xd = blk;
    *yd = (D == 2) ? blk + n : NULL;
}

/* Public: evaluate R (and optionally grad / packed Hessian) at n_theta points
 * of ONE event, all in FP64. theta is n_theta x n_par. */
void oracle_response(int D, int n_planes, const float* plane_z, int64_t n_hits,
                     const float* x, const float* y, const int32_t* plane,
                     int64_t n_theta, const double* theta, double sigma,
                     double* R, double* grad, double* hess)
{
    const int np = 2 * D;
    double pz[64];
    double* pzh = n_planes <= 64 ? pz : (double*)malloc(sizeof(double) * (size_t)n_planes);
    for (int p = 0; p < n_planes; ++p) pzh[p] = (double)plane_z[p];
    double *xd, *yd;
    widen(D, n_hits, x, y, &xd, &yd);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n_theta; ++i) {
        double Hf[MAXP * MAXP], gl[MAXP], Rl;
        response_one(D, pzh, n_hits, xd, yd, plane, theta + i * np, sigma, &Rl, gl, Hf);
        R[i] = Rl;
        if (grad) for (int a = 0; a < np; ++a) grad[i * np + a] = gl[a];
        if (hess) {
            int q = 0;
            for (int a = 0; a < np; ++a)
                for (int b = a; b < np; ++b) hess[i * (np * (np + 1) / 2) + q++] = Hf[a * np + b];
        }
    }
    free(xd);
    if (pzh != pz) free(pzh);
}

/* ------------------------------------------------------------------------- */
/* Truncated Newton direction (Section 3 names Truncated Newton as the update;
 * the inner solve is the line-search Newton-CG of Nocedal & Wright, Ch. 7),
 * applied to f = -R in scaled coordinates theta~ = Dscale*theta.
 *   b = Dscale^-1 g,  A = -Dscale^-1 H Dscale^-1
 *   CG on A p = b from p = 0, at most n_par iterations, stopping once the
 *   residual is below cg_rtol*|b| (a relative forcing term: the textbook
 *   min(0.5, sqrt(|b|)) |b| depends on the units of R and truncates after one
 *   iteration here, since |b| >> 1 in R per mm).
 *   Negative or zero curvature on the first direction: steepest ascent
 *   normalised to one bandwidth, p = sigma * b/|b|; on a later direction:
 *   the current iterate.
 *   The scaled step is capped at cap*sigma.
 * Returns the unscaled direction p = Dscale^-1 p~, the scaled length |p~|,
 * and *negcurv = 1 if a non-positive curvature was met.                     */
void oracle_newton_cg(int np, const double* g, const double* H, const double* dscale,
                      double sigma, double cap, double* p_out, double* pnorm_out, int* negcurv)
{
    double b[MAXP], A[MAXP][MAXP];
    for (int a = 0; a < np; ++a) b[a] = g[a] / dscale[a];
    for (int a = 0; a < np; ++a)
        for (int c = 0; c < np; ++c) A[a][c] = -H[a * np + c] / (dscale[a] * dscale[c]);
    double bn = 0.0;
    for (int a = 0; a < np; ++a) bn += b[a] * b[a];
    bn = sqrt(bn);
    double p[MAXP] = {0};
    *negcurv = 0;
    if (bn > 0.0) {
        const double eps = CG_RTOL * bn;
        double zv[MAXP] = {0}, r[MAXP], d[MAXP];
        for (int a = 0; a < np; ++a) { r[a] = b[a]; d[a] = b[a]; }
        int done = 0;
        for (int k = 0; k < np && !done; ++k) {
            double Ad[MAXP], dAd = 0.0, rr = 0.0;
            for (int a = 0; a < np; ++a) {
                Ad[a] = 0.0;
                for (int c = 0; c < np; ++c) Ad[a] += A[a][c] * d[c];
            }
            for (int a = 0; a < np; ++a) { dAd += d[a] * Ad[a]; rr += r[a] * r[a]; }
            if (dAd <= 0.0) {
                *negcurv = 1;
                if (k == 0) for (int a = 0; a < np; ++a) p[a] = sigma * b[a] / bn;
                else for (int a = 0; a < np; ++a) p[a] = zv[a];
                done = 1;
                break;
            }
            const double alpha = rr / dAd;
            double rr_new = 0.0;
            for (int a = 0; a < np; ++a) {
                zv[a] += alpha * d[a];
                r[a] -= alpha * Ad[a];
                rr_new += r[a] * r[a];
            }
            if (sqrt(rr_new) < eps) {
                for (int a = 0; a < np; ++a) p[a] = zv[a];
                done = 1;
                break;
            }
            const double beta = rr_new / rr;
            for (int a = 0; a < np; ++a) d[a] = r[a] + beta * d[a];
        }
        if (!done) for (int a = 0; a < np; ++a) p[a] = zv[a];
    }
    double pn = 0.0;
    for (int a = 0; a < np; ++a) pn += p[a] * p[a];
    pn = sqrt(pn);
    if (pn > cap * sigma) {
        const double s = cap * sigma / pn;
        for (int a = 0; a < np; ++a) p[a] *= s;
        pn = cap * sigma;
    }
    for (int a = 0; a < np; ++a) p_out[a] = p[a] / dscale[a];
    *pnorm_out = pn;
}

/* Cholesky solve of A delta = b for a small SPD A (FP64).  Returns 0 when A
 * is not positive definite. */
static int chol_solve(int n, const double* A, const double* b, double* x)
{
    double L[MAXP][MAXP] = {{0}};
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0)) return 0;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    double t[MAXP];
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * t[k];
        t[i] = s / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = t[i];
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return 1;
}

/* Scaling matrix of the Newton-CG step: unit scale on offsets, z_ref (the RMS
 * plane coordinate) on slopes, so every scaled component is a displacement
 * in length units at z_ref. */
static double z_rms(int n_planes, const double* pz)
{
    double s = 0.0;
    for (int p = 0; p < n_planes; ++p) s += pz[p] * pz[p];
    return sqrt(s / (double)n_planes);
}

static void make_dscale(int D, double zref, double* ds)
{
    if (D == 2) { ds[0] = 1.0; ds[1] = 1.0; ds[2] = zref; ds[3] = zref; }
    else { ds[0] = 1.0; ds[1] = zref; }
}

/* FP64 Newton polish at sigma_final: n_iter times, if -H is positive definite
 * theta += (-H)^-1 g; the first slope_iters iterations (D = 2) solve on the
 * slope block only, offsets held.  Reports R of the last evaluation, the
 * scaled length of the last step and whether -H (or its slope block) was
 * positive definite there. */
static void polish_one(int D, const double* pz, const double* ds, int64_t n, const double* x,
                       const double* y, const int32_t* pl, double* th, double sigma, int n_iter,
                       int slope_iters, double* R_out, double* step_out, int* pd_out)
{
    const int np = 2 * D;
    double R = 0.0, step = INFINITY;
    int pd = 0;
    for (int it = 0; it < n_iter; ++it) {
        double g[MAXP], H[MAXP * MAXP], A[MAXP * MAXP], dl[MAXP];
        response_one(D, pz, n, x, y, pl, th, sigma, &R, g, H);
        if (D == 2 && it < slope_iters) {
            /* offsets held: the Newton system of the slope block */
            const double As[4] = {-H[2 * np + 2], -H[2 * np + 3], -H[3 * np + 2], -H[3 * np + 3]};
            const double gs[2] = {g[2], g[3]};
            double ds2[2];
            pd = chol_solve(2, As, gs, ds2);
            dl[0] = 0.0; dl[1] = 0.0; dl[2] = ds2[0]; dl[3] = ds2[1];
        } else {
            for (int a = 0; a < np * np; ++a) A[a] = -H[a];
            pd = chol_solve(np, A, g, dl);
        }
        if (pd) {
            double s = 0.0;
            for (int a = 0; a < np; ++a) {
                th[a] += dl[a];
                s += (ds[a] * dl[a]) * (ds[a] * dl[a]);
            }
            step = sqrt(s);
        } else {
            step = INFINITY;
        }
    }
    *R_out = R;
    *step_out = step;
    *pd_out = pd;
}

/* BFGS update of an inverse-Hessian model B (n x n, row-major, in place)
 * with step s and gradient change y, s.y > 0 (Nocedal & Wright, Ch. 6):
 * B <- (I - rho s y^T) B (I - rho y s^T) + rho s s^T,  rho = 1 / (y.s). */
void oracle_bfgs_update(int n, double* B, const double* s, const double* y)
{
    double sy = 0.0;
    for (int a = 0; a < n; ++a) sy += s[a] * y[a];
    const double rho = 1.0 / sy;
    double E[MAXP * MAXP], Bn[MAXP * MAXP];
    for (int a = 0; a < n; ++a)
        for (int c = 0; c < n; ++c) E[a * n + c] = (a == c ? 1.0 : 0.0) - rho * s[a] * y[c];
    for (int a = 0; a < n; ++a)
        for (int c = 0; c < n; ++c) {
            double v = 0.0;
            for (int k = 0; k < n; ++k)
                for (int l = 0; l < n; ++l) v += E[a * n + k] * B[k * n + l] * E[c * n + l];
            Bn[a * n + c] = v + rho * s[a] * s[c];
        }
    for (int a = 0; a < n * n; ++a) B[a] = Bn[a];
}

/* One multi-start trajectory (Algorithm 1, the loop over j for a fixed i):
 * seeds are independent, so a seed's whole trajectory can run before the
 * next seed's without changing any result.
 *   for s = 1 .. n_sigma + n_final_steps:
 *     sigma_s = sigma[s] for the continuation stages, then sigma_final
 *     (R, g, H) at theta;  p = the update rule's direction: Newton-CG
 *       (truncated Newton, Section 3's choice), the normalised gradient, or
 *       BFGS on the scaled gradient restarted whenever sigma changes (other
 *       methods the paper reports examining)
 *     if the scaled Newton step is small (no negative curvature and
 *       |p~| <= small_step_sigmas*sigma_s): theta += p
 *     else backtracking: first alpha in 1, 1/2, 1/4, .. (ls_trials values)
 *       with R(theta + alpha p) >= R + c1*alpha*g.p; none -> theta kept,
 *       the seed is flagged stalled.
 *   then the FP64 polish at sigma_final.
 * Output: theta, R at the last polish evaluation, flags, and the number of
 * R-only evaluations spent in line searches. */
static void ascend_one(int D, const double* pz, double zref, int64_t n, const double* x,
                       const double* y, const int32_t* pl, const oracle_params* P,
                       double* th, double* R_out, int32_t* flags_out, int32_t* n_reval_out)
{
    const int np = 2 * D;
    double ds[MAXP];
    make_dscale(D, zref, ds);
    const int n_steps = P->n_sigma + P->n_final_steps;
    int32_t flags = 0, n_reval = 0;
    /* state of the quasi-Newton rule (scaled coordinates): inverse-Hessian
     * model, gradient and accepted step of the previous update */
    double Bm[MAXP * MAXP] = {0}, b_prev[MAXP] = {0}, s_prev[MAXP] = {0}, sig_prev = 0.0;
    for (int s = 0; s < n_steps; ++s) {
        const double sig = (double)(s < P->n_sigma ? P->sigma[s] : P->sigma_final);
        double R, g[MAXP], H[MAXP * MAXP], p[MAXP], pn;
        int neg;
        response_one(D, pz, n, x, y, pl, th, sig, &R, g, H);
        const int slope_only = D == 2 && s < P->n_slope_steps;
        if (P->update != 0) {
            /* first-order and quasi-Newton rules in the scaled coordinates */
            double b[MAXP], q[MAXP], bn = 0.0;
            for (int a = 0; a < np; ++a) b[a] = (slope_only && a < 2) ? 0.0 : g[a] / ds[a];
            for (int a = 0; a < np; ++a) bn += b[a] * b[a];
            bn = sqrt(bn);
            if (P->update == 1 || s == 0 || sig != sig_prev) {
                /* normalised gradient step of one bandwidth; BFGS (re)starts here
                 * with the inverse-Hessian model (sigma / |b|) I */
                for (int a = 0; a < np * np; ++a) Bm[a] = 0.0;
                for (int a = 0; a < np; ++a) Bm[a * np + a] = bn > 0.0 ? sig / bn : 0.0;
            } else {
                /* BFGS update of the inverse Hessian of f = -R with the last
                 * step s~ and the change of grad f, y = -(b - b_prev); skipped
                 * unless s~.y > 0 */
                double yv[MAXP], sy = 0.0;
                for (int a = 0; a < np; ++a) { yv[a] = -(b[a] - b_prev[a]); sy += s_prev[a] * yv[a]; }
                if (sy > 0.0) oracle_bfgs_update(np, Bm, s_prev, yv);
            }
            for (int a = 0; a < np; ++a) {
                double v = 0.0;
                for (int c2 = 0; c2 < np; ++c2) v += Bm[a * np + c2] * b[c2];
                q[a] = v;
            }
            double qn = 0.0;
            for (int a = 0; a < np; ++a) qn += q[a] * q[a];
            qn = sqrt(qn);
            const double lim = (double)P->step_cap_sigmas * sig;
            if (qn > lim) { for (int a = 0; a < np; ++a) q[a] *= lim / qn; qn = lim; }
            for (int a = 0; a < np; ++a) { p[a] = q[a] / ds[a]; b_prev[a] = b[a]; s_prev[a] = 0.0; }
            pn = qn;
            neg = 0;
        } else if (slope_only) {
            /* offsets held at their current values: Newton-CG on the slope block */
            const double gs[2] = {g[2], g[3]};
            const double Hs[4] = {H[2 * np + 2], H[2 * np + 3], H[3 * np + 2], H[3 * np + 3]};
            const double dss[2] = {ds[2], ds[3]};
            double ps[2];
            oracle_newton_cg(2, gs, Hs, dss, sig, (double)P->step_cap_sigmas, ps, &pn, &neg);
            p[0] = 0.0; p[1] = 0.0; p[2] = ps[0]; p[3] = ps[1];
        } else {
            oracle_newton_cg(np, g, H, ds, sig, (double)P->step_cap_sigmas, p, &pn, &neg);
        }
        sig_prev = sig;
        if (neg) flags |= OR_NEGCURV;
        if (!neg && pn <= (double)P->small_step_sigmas * sig) {
            for (int a = 0; a < np; ++a) { th[a] += p[a]; s_prev[a] = ds[a] * p[a]; }
            continue;
        }
        double gp = 0.0;
        for (int a = 0; a < np; ++a) gp += g[a] * p[a];
        int accepted = 0;
        double alpha = 1.0;
        for (int t = 0; t < P->ls_trials; ++t, alpha *= 0.5) {
            double tt[MAXP];
            for (int a = 0; a < np; ++a) tt[a] = th[a] + alpha * p[a];
            const double Rt = response_only(D, pz, n, x, y, pl, tt, sig);
            ++n_reval;
            if (Rt >= R + (double)P->armijo_c1 * alpha * gp) {
                for (int a = 0; a < np; ++a) { th[a] = tt[a]; s_prev[a] = ds[a] * alpha * p[a]; }
                accepted = 1;
                break;
            }
        }
        if (!accepted) flags |= OR_STALLED;
    }
    double R, step;
    int pd;
    /* n_slope_steps counts the steps, then the polish iterations: a count past
     * the steps holds the offsets in that many polish iterations too */
    const int slope_iters = P->n_slope_steps > n_steps ? P->n_slope_steps - n_steps : 0;
    polish_one(D, pz, ds, n, x, y, pl, th, (double)P->sigma_final, P->n_polish, slope_iters, &R, &step, &pd);
    if (!pd) flags |= OR_NOT_PD;
    if (pd && step <= (double)P->conv_tol * (double)P->sigma_final) flags |= OR_CONVERGED;
    *R_out = R;
    *flags_out = flags;
    *n_reval_out = n_reval;
}

/* Lattice seed i (Algorithm 1, first loop; the prior is a cell-centred
 * lattice over a box): value = FP32 rounding of lo + (j + 1/2)(hi - lo)/n,
 * formed in FP64; dimension 0 is the slow index.
 *   D = 2: dims (tx, ty), x0 = y0 = 0;   D = 1: dims (tx, x0). */
static void lattice_seed(int D, const oracle_params* P, int64_t i, double* th)
{
    const int64_t n1 = P->lattice_n[1];
    const int64_t j0 = i / n1, j1 = i % n1;
    double v[2];
    for (int d = 0; d < 2; ++d) {
        const int64_t j = d == 0 ? j0 : j1;
        const double lo = (double)P->lattice_lo[d], hi = (double)P->lattice_hi[d];
        v[d] = (double)(float)(lo + ((double)j + 0.5) * (hi - lo) / (double)P->lattice_n[d]);
    }
    if (D == 2) { th[0] = 0.0; th[1] = 0.0; th[2] = v[0]; th[3] = v[1]; }
    else { th[0] = v[1]; th[1] = v[0]; }
}

/* Distance used to cluster two solutions: the largest in-plane separation of
 * the two lines over the detector's end planes (the separation is linear in
 * z, so its maximum over the detector sits at an end plane). */
static double track_distance(int D, const double* a, const double* b, double z_first, double z_last)
{
    double d = 0.0;
    const double zz[2] = {z_first, z_last};
    for (int q = 0; q < 2; ++q) {
        if (D == 2) {
            const double dx = fabs((a[0] - b[0]) + (a[2] - b[2]) * zz[q]);
            const double dy = fabs((a[1] - b[1]) + (a[3] - b[3]) * zz[q]);
            d = fmax(d, fmax(dx, dy));
        } else {
            d = fmax(d, fabs((a[0] - b[0]) + (a[1] - b[1]) * zz[q]));
        }
    }
    return d;
}

typedef struct { double R; int64_t idx; } cand_t;

static int cand_cmp(const void* pa, const void* pb)
{
    const cand_t* a = (const cand_t*)pa;
    const cand_t* b = (const cand_t*)pb;
    if (a->R > b->R) return -1;
    if (a->R < b->R) return 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

/* Algorithm 1, last two steps, for one event: keep converged solutions with
 * R >= R0; visit them by decreasing R (ties: lower seed index first); each
 * joins the first existing cluster whose leader lies within d_merge, else it
 * founds a new cluster.  A leader is therefore the highest-response solution
 * of its cluster.  Returns the number of clusters; out_* receive the leaders
 * in creation order. */
int64_t oracle_merge(int D, int64_t n_seeds, const double* theta, const double* R,
                     const int32_t* flags, double R0, double d_merge, double z_first,
                     double z_last, int64_t* out_leader, int32_t* out_members)
{
    const int np = 2 * D;
    cand_t* c = (cand_t*)malloc(sizeof(cand_t) * (size_t)(n_seeds > 0 ? n_seeds : 1));
    int64_t nc = 0;
    for (int64_t i = 0; i < n_seeds; ++i)
        if ((flags[i] & OR_CONVERGED) && R[i] >= R0) { c[nc].R = R[i]; c[nc].idx = i; ++nc; }
    qsort(c, (size_t)nc, sizeof(cand_t), cand_cmp);
    int64_t nl = 0;
    for (int64_t k = 0; k < nc; ++k) {
        const double* t = theta + c[k].idx * np;
        int64_t join = -1;
        for (int64_t l = 0; l < nl; ++l) {
            if (track_distance(D, t, theta + out_leader[l] * np, z_first, z_last) <= d_merge) {
                join = l;
                break;
            }
        }
        if (join >= 0) {
            out_members[join] += 1;
        } else {
            out_leader[nl] = c[k].idx;
            out_members[nl] = 1;
            ++nl;
        }
    }
    free(c);
    return nl;
}

/* Algorithm 1 end to end over a batch.  Seeds: the lattice of P when
 * seeds == NULL, else explicit seeds (seed_offsets[n_events+1], n_par
 * doubles each).  Per-seed outputs (seed_theta, seed_R, seed_flags,
 * seed_nreval) are indexed by global seed number and may be NULL.  Tracks:
 * event e's clusters go to slots trk_offsets[e] .. trk_offsets[e+1]-1, packed
 * in event order; the caller sizes trk_* for the total seed count.
 * n_threads <= 0 uses the OpenMP default. */
int oracle_find_tracks(int D, int n_planes, const float* plane_z, int64_t n_events,
                       const int64_t* event_offsets, const float* x, const float* y,
                       const int32_t* plane, const oracle_params* P, const double* seeds,
                       const int64_t* seed_offsets, double* seed_theta, double* seed_R,
                       int32_t* seed_flags, int32_t* seed_nreval, double* trk_theta,
                       double* trk_R, int32_t* trk_members, int64_t* trk_seed,
                       int64_t* trk_offsets, int n_threads)
{
    const int np = 2 * D;
    double pz[256];
    if (n_planes > 256 || n_planes < 1) return -1;
    for (int p = 0; p < n_planes; ++p) pz[p] = (double)plane_z[p];
    const double zref = z_rms(n_planes, pz);
    double zmin = pz[0], zmax = pz[0];
    for (int p = 1; p < n_planes; ++p) { zmin = fmin(zmin, pz[p]); zmax = fmax(zmax, pz[p]); }
    const int64_t lat = (int64_t)P->lattice_n[0] * (int64_t)P->lattice_n[1];

    int64_t* soff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_events + 1));
    soff[0] = 0;
    for (int64_t e = 0; e < n_events; ++e)
        soff[e + 1] = soff[e] + (seeds ? seed_offsets[e + 1] - seed_offsets[e] : lat);
    const int64_t n_seeds = soff[n_events];

    double* th = (double*)malloc(sizeof(double) * (size_t)(n_seeds > 0 ? n_seeds : 1) * np);
    double* Rs = (double*)malloc(sizeof(double) * (size_t)(n_seeds > 0 ? n_seeds : 1));
    int32_t* fl = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_seeds > 0 ? n_seeds : 1));
    int32_t* nr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_seeds > 0 ? n_seeds : 1));
    const int64_t total_hits = event_offsets[n_events];
    double *xd, *yd;
    widen(D, total_hits, x, y, &xd, &yd);

#ifdef _OPENMP
    const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
#endif
    for (int64_t gs = 0; gs < n_seeds; ++gs) {
        int64_t e = 0, lo = 0, hi = n_events;  /* event of global seed gs */
        while (hi - lo > 1) { const int64_t m = (lo + hi) / 2; if (soff[m] <= gs) lo = m; else hi = m; }
        e = lo;
        const int64_t i = gs - soff[e];
        double* t = th + gs * np;
        if (seeds) for (int a = 0; a < np; ++a) t[a] = seeds[(seed_offsets[e] + i) * np + a];
        else lattice_seed(D, P, i, t);
        const int64_t h0 = event_offsets[e], nh = event_offsets[e + 1] - h0;
        ascend_one(D, pz, zref, nh, xd + h0, yd ? yd + h0 : NULL, plane + h0, P, t, &Rs[gs], &fl[gs], &nr[gs]);
    }

    /* merge per event (independent events in parallel), then pack */
    int64_t* ldr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_seeds > 0 ? n_seeds : 1));
    int32_t* mem = (int32_t*)calloc((size_t)(n_seeds > 0 ? n_seeds : 1), sizeof(int32_t));
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_events > 0 ? n_events : 1));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int64_t e = 0; e < n_events; ++e) {
        const int64_t s0 = soff[e], ns = soff[e + 1] - s0;
        cnt[e] = oracle_merge(D, ns, th + s0 * np, Rs + s0, fl + s0, (double)P->R0,
                              (double)P->d_merge, zmin, zmax, ldr + s0, mem + s0);
    }
    trk_offsets[0] = 0;
    for (int64_t e = 0; e < n_events; ++e) {
        const int64_t s0 = soff[e];
        int64_t o = trk_offsets[e];
        for (int64_t l = 0; l < cnt[e]; ++l, ++o) {
            const int64_t gs = s0 + ldr[s0 + l];
            for (int a = 0; a < np; ++a) trk_theta[o * np + a] = th[gs * np + a];
            trk_R[o] = Rs[gs];
            trk_members[o] = mem[s0 + l];
            trk_seed[o] = ldr[s0 + l];
        }
        trk_offsets[e + 1] = o;
    }
    if (seed_theta) memcpy(seed_theta, th, sizeof(double) * (size_t)n_seeds * np);
    if (seed_R) memcpy(seed_R, Rs, sizeof(double) * (size_t)n_seeds);
    if (seed_flags) memcpy(seed_flags, fl, sizeof(int32_t) * (size_t)n_seeds);
    if (seed_nreval) memcpy(seed_nreval, nr, sizeof(int32_t) * (size_t)n_seeds);
    free(cnt); free(mem); free(ldr); free(xd); free(nr); free(fl); free(Rs); free(th); free(soff);
    return 0;
}

/* Newton polish of n arbitrary points of one event (used to refine the
 * brute-force grid maxima): see polish_one. */
void oracle_polish(int D, int n_planes, const float* plane_z, int64_t n_hits, const float* x,
                   const float* y, const int32_t* plane, int64_t n_theta, double* theta,
                   double sigma, int n_iter, double* R_out, double* step_out, int32_t* pd_out)
{
    const int np = 2 * D;
    double pz[256];
    for (int p = 0; p < n_planes && p < 256; ++p) pz[p] = (double)plane_z[p];
    double ds[MAXP];
    make_dscale(D, z_rms(n_planes, pz), ds);
    double *xd, *yd;
    widen(D, n_hits, x, y, &xd, &yd);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n_theta; ++i) {
        int pd;
        polish_one(D, pz, ds, n_hits, xd, yd, plane, theta + i * np, sigma, n_iter, 0, &R_out[i], &step_out[i], &pd);
        pd_out[i] = pd;
    }
    free(xd);
}

/* The lattice seeds as the oracle forms them (for tests of the seeding). */
void oracle_lattice(int D, const oracle_params* P, double* out)
{
    const int64_t n = (int64_t)P->lattice_n[0] * P->lattice_n[1];
    for (int64_t i = 0; i < n; ++i) lattice_seed(D, P, i, out + i * 2 * D);
}

/* ------------------------------------------------------------------------- */
/* The plain Artificial Retina that the method replaces (Section 2, the four
 * usual steps of grid-based AR algorithms):
 *   1. a parameter grid: the cell-centred lattice of lattice_seed over the
 *      box of P (same FP32 cell centres, slow index first);
 *   2. the response of Eq. (1) at every cell, at bandwidth sigma;
 *   3. groups of high-response cells: read as the strict local maxima of the
 *      grid response over the up to 8 neighbouring cells inside the grid,
 *      with R >= R0 (a cell whose neighbour has an equal response is not a
 *      maximum);
 *   4. one estimate per cluster: read as the response-weighted mean of the
 *      cell centres of the maximum's 3 x 3 neighbourhood (cells inside the
 *      grid only).
 * One event.  Outputs: R_grid[n0 * n1] (may be NULL); the peaks in cell
 * order: peak_cell, peak_theta (n_par doubles; the parameters the grid does
 * not span are 0), peak_R (the maximum's response), peak_members (cells of
 * the neighbourhood with R >= R0, the maximum included).  At most max_peaks
 * are written; the return value is the number of peaks found.              */
int64_t oracle_grid_search(int D, int n_planes, const float* plane_z, int64_t n_hits, const float* x,
                           const float* y, const int32_t* plane, const oracle_params* P, double sigma,
                           double R0, double* R_grid, int64_t max_peaks, int64_t* peak_cell,
                           double* peak_theta, double* peak_R, int32_t* peak_members, int n_threads)
{
    const int np = 2 * D;
    double pz[256];
    if (n_planes > 256 || n_planes < 1) return -1;
    for (int p = 0; p < n_planes; ++p) pz[p] = (double)plane_z[p];
    const int64_t n0 = P->lattice_n[0], n1 = P->lattice_n[1], nc = n0 * n1;
    double* G = (double*)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    double *xd, *yd;
    widen(D, n_hits, x, y, &xd, &yd);
#ifdef _OPENMP
    const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
#endif
    for (int64_t c = 0; c < nc; ++c) {
        double th[MAXP];
        lattice_seed(D, P, c, th);
        G[c] = response_only(D, pz, n_hits, xd, yd, plane, th, sigma);
    }
    int64_t n_peaks = 0;
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t i0 = c / n1, i1 = c % n1;
        const double Rc = G[c];
        if (!(Rc >= R0)) continue;
        int is_max = 1;
        for (int d0 = -1; d0 <= 1 && is_max; ++d0)
            for (int d1 = -1; d1 <= 1; ++d1) {
                const int64_t j0 = i0 + d0, j1 = i1 + d1;
                if ((d0 == 0 && d1 == 0) || j0 < 0 || j0 >= n0 || j1 < 0 || j1 >= n1) continue;
                if (!(Rc > G[j0 * n1 + j1])) { is_max = 0; break; }
            }
        if (!is_max) continue;
        if (n_peaks < max_peaks) {
            double wsum = 0.0, tsum[MAXP] = {0};
            int32_t members = 0;
            for (int d0 = -1; d0 <= 1; ++d0)
                for (int d1 = -1; d1 <= 1; ++d1) {
                    const int64_t j0 = i0 + d0, j1 = i1 + d1;
                    if (j0 < 0 || j0 >= n0 || j1 < 0 || j1 >= n1) continue;
                    const double w = G[j0 * n1 + j1];
                    double th[MAXP];
                    lattice_seed(D, P, j0 * n1 + j1, th);
                    wsum += w;
                    for (int a = 0; a < np; ++a) tsum[a] += w * th[a];
                    if (w >= R0) ++members;
                }
            double tc[MAXP];
            lattice_seed(D, P, c, tc);
            peak_cell[n_peaks] = c;
            for (int a = 0; a < np; ++a) peak_theta[n_peaks * np + a] = wsum > 0.0 ? tsum[a] / wsum : tc[a];
            peak_R[n_peaks] = Rc;
            peak_members[n_peaks] = members;
        }
        ++n_peaks;
    }
    if (R_grid) memcpy(R_grid, G, sizeof(double) * (size_t)nc);
    free(xd);
    free(G);
    return n_peaks;
}

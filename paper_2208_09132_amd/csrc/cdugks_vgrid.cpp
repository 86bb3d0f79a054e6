// Velocity grid fitted to a state: the paper's criterion for its fixed grid
// (Sec. 5: fine enough to resolve the mass, wide enough to hold all of it,
// both to a chosen integration error), applied to the current moments so
// that a problem can be refit (cdugks_regrid) as it evolves.  Host code only.
#include "cdugks.h"
#include "cdugks_host.h"

#include <algorithm>
#include <cmath>

using namespace cdg;

int cdugks_fit_velocity(const cdugks_space* space, const cdugks_params* params, const double* rho,
                        const double* u, const double* T, double tol, int quadrature, cdugks_velocity* out) {
    if (!space || !params || !rho || !u || !T || !out) return fail(CDUGKS_ERR_INVALID, "null argument");
    const int D = space->dim;
    if (D < 1 || D > 3) return fail(CDUGKS_ERR_INVALID, "dim must be 1, 2 or 3");
    if (!(tol > 0.0 && tol < 1.0)) return fail(CDUGKS_ERR_INVALID, "tol must lie in (0, 1)");
    if (quadrature != CDUGKS_QUAD_TRAPEZOID && quadrature != CDUGKS_QUAD_BOOLE)
        return fail(CDUGKS_ERR_INVALID, "unknown quadrature rule");
    long long N = 1;
    for (int d = 0; d < D; ++d) {
        if (space->n[d] < 1) return fail(CDUGKS_ERR_INVALID, "n[%d] must be >= 1", d);
        N *= space->n[d];
    }
    const double R = params->R > 0.0 ? params->R : 0.5;
    // width: u_d +- k sigma in every cell, sigma = sqrt(R T), with k such that
    // the normal tail beyond k sigma on one side, at most exp(-k^2/2)/2, is
    // at most tol/2
    const double k = std::sqrt(2.0 * std::log(1.0 / tol));
    // spacing: the trapezoid rule on a Gaussian of deviation sigma errs by
    // about 2 exp(-2 pi^2 sigma^2 / h^2) (its first aliasing term); at most
    // tol for the narrowest cell
    double smin = HUGE_VAL;
    double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (long long c = 0; c < N; ++c) {
        if (!(rho[c] > 0.0) || !(T[c] > 0.0) || !std::isfinite(T[c]))
            return fail(CDUGKS_ERR_INVALID, "non-physical moments at cell %lld", c);
        const double s = std::sqrt(R * T[c]);
        smin = std::min(smin, s);
        for (int d = 0; d < D; ++d) {
            const double ud = u[(long long)d * N + c];
            if (!std::isfinite(ud)) return fail(CDUGKS_ERR_INVALID, "u[%d][%lld] is not finite", d, c);
            lo[d] = std::min(lo[d], ud - k * s);
            hi[d] = std::max(hi[d], ud + k * s);
        }
    }
    const double h = M_PI * smin * std::sqrt(2.0) / std::sqrt(std::log(2.0 / tol));
    for (int d = 0; d < 3; ++d) {
        if (d >= D) {
            out->nv[d] = 1;
            out->vmin[d] = out->vmax[d] = 0.0;
            continue;
        }
        long long nv = (long long)std::ceil((hi[d] - lo[d]) / h) + 1;
        nv = std::max<long long>(nv, 2);
        if (quadrature == CDUGKS_QUAD_BOOLE) nv = (nv - 1 + 3) / 4 * 4 + 1;  // 4n + 1 nodes
        out->nv[d] = nv;
        out->vmin[d] = lo[d];
        out->vmax[d] = hi[d];
    }
    out->quadrature = quadrature;
    return CDUGKS_OK;
}

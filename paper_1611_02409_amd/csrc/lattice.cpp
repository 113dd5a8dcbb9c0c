// Host-side lattice constants and relaxation parameters.
//
// Weights and scale factor: a velocity set built on Gauss-Hermite quadrature
// (Section VI.A) must integrate the even monomials xi_x^2a xi_y^2b (xi_z^2c)
// of the unit Gaussian exactly up to its degree.  With xi = r c and x = r^2,
// every condition is linear in the shell weights for fixed x.  Here the
// first nshell conditions fix the weights by a linear solve at given x, the
// remaining condition becomes a scalar equation F(x) = 0, and x is found by
// scanning for a bracket with all weights positive and then bisecting in long
// double.
#include "lattice.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>

#include "../../include/esbgk.h"

namespace esbgk {

namespace {

template <class L>
void fill_velocities(LatticeConsts &lc) {
    lc.D = L::D;
    lc.Q = L::Q;
    lc.NP = L::NP;
    lc.nshell = L::NSHELL;
    lc.reach = L::REACH;
    for (int d = 0; d < 3; d++) lc.c[0][d] = 0;
    lc.shell_of[0] = 0;
    for (int p = 0; p < L::NP; p++) {
        for (int d = 0; d < 3; d++) {
            lc.c[2 * p + 1][d] = L::P[p].c[d];
            lc.c[2 * p + 2][d] = -L::P[p].c[d];
        }
        lc.shell_of[2 * p + 1] = lc.shell_of[2 * p + 2] = L::P[p].shell;
    }
}

long double dfact(int n) {
    long double v = 1;
    for (; n > 1; n -= 2) v *= n;
    return v;
}

// Moment conditions: exponent triples (a, b, c) of xi_x^2a xi_y^2b xi_z^2c.
const int COND2[9][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {2, 0, 0}, {2, 1, 0},
                         {3, 0, 0}, {2, 2, 0}, {3, 1, 0}, {4, 0, 0}};
const int COND3[7][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {2, 0, 0}, {1, 1, 1}, {3, 0, 0}, {2, 1, 0}};

struct System {
    int ns = 0, nc = 0;
    long double M[9][8] = {};   // M[k][s]: sum over shell s of the integer monomial
    int deg[9] = {};
    long double rhs[9] = {};
};

System build_system(const LatticeConsts &lc) {
    System S;
    S.ns = lc.nshell;
    S.nc = lc.D == 2 ? 9 : 7;
    for (int k = 0; k < S.nc; k++) {
        const int *e = lc.D == 2 ? COND2[k] : COND3[k];
        S.deg[k] = e[0] + e[1] + e[2];
        S.rhs[k] = dfact(2 * e[0] - 1) * dfact(2 * e[1] - 1) * dfact(2 * e[2] - 1);
        for (int i = 0; i < lc.Q; i++) {
            long double m = 1;
            for (int d = 0; d < 3; d++)
                for (int t = 0; t < 2 * e[d]; t++) m *= lc.c[i][d];
            S.M[k][lc.shell_of[i]] += m;
        }
    }
    return S;
}

// Weights from the first ns conditions at x = r^2 (Gauss-Jordan, partial
// pivoting); returns the residual of the last condition, or NAN if singular.
long double weights_at(const System &S, long double x, long double *w) {
    const int n = S.ns;
    long double A[8][9];
    for (int k = 0; k < n; k++) {
        long double xp = powl(x, S.deg[k]);
        for (int s = 0; s < n; s++) A[k][s] = S.M[k][s] * xp;
        A[k][n] = S.rhs[k];
    }
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
        if (fabsl(A[piv][col]) < 1e-200L) return NAN;
        if (piv != col)
            for (int j = 0; j <= n; j++) std::swap(A[piv][j], A[col][j]);
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            long double f = A[r][col] / A[col][col];
            for (int j = col; j <= n; j++) A[r][j] -= f * A[col][j];
        }
    }
    for (int s = 0; s < n; s++) w[s] = A[s][n] / A[s][s];
    long double res = -S.rhs[n];
    long double xp = powl(x, S.deg[n]);
    for (int s = 0; s < n; s++) res += S.M[n][s] * w[s] * xp;
    return res;
}

bool all_positive(const long double *w, int n) {
    for (int s = 0; s < n; s++)
        if (!(w[s] > 0)) return false;
    return true;
}

bool solve(LatticeConsts &lc) {
    System S = build_system(lc);
    long double w[8], lo = 0, hi = 0;
    long double prev_x = 0.3L, prev_f = weights_at(S, prev_x, w);
    bool found = false;
    for (long double x = 0.31L; x < 6.0L; x += 0.01L) {
        long double f = weights_at(S, x, w);
        if (!std::isnan((double)f) && !std::isnan((double)prev_f) && (f > 0) != (prev_f > 0)) {
            long double wm[8];
            weights_at(S, 0.5L * (x + prev_x), wm);
            if (all_positive(wm, S.ns)) {
                lo = prev_x;
                hi = x;
                found = true;
                break;
            }
        }
        prev_x = x;
        prev_f = f;
    }
    if (!found) return false;
    long double flo = weights_at(S, lo, w);
    for (int it = 0; it < 200; it++) {
        long double mid = 0.5L * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        long double fm = weights_at(S, mid, w);
        if ((fm > 0) == (flo > 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    long double x = 0.5L * (lo + hi);
    weights_at(S, x, w);
    if (!all_positive(w, S.ns)) return false;
    lc.r = (double)sqrtl(x);
    for (int s = 0; s < S.ns; s++) {
        lc.wshell[s] = (double)w[s];
        lc.scale_exp[s] = (int)std::floor(std::log2(1.0 / lc.wshell[s]));
    }
    return true;
}

std::mutex g_mu;
LatticeConsts g_cache[3];
bool g_ready[3] = {false, false, false};

}  // namespace

bool lattice_consts(int D, int Q, LatticeConsts &out) {
    int slot;
    if (D == 2 && Q == 37) slot = 0;
    else if (D == 2 && Q == 33) slot = 1;
    else if (D == 3 && Q == 39) slot = 2;
    else return false;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ready[slot]) {
        LatticeConsts lc;
        if (slot == 0) fill_velocities<LatD2Q37>(lc);
        else if (slot == 1) fill_velocities<LatD2Q33>(lc);
        else fill_velocities<LatD3Q39>(lc);
        if (!solve(lc)) return false;
        g_cache[slot] = lc;
        g_ready[slot] = true;
    }
    out = g_cache[slot];
    return true;
}

int derive_params(int D, int Nf, double Pr, double tau, double kappa, double out[4], char *err, size_t errlen) {
    if (!(D == 2 || D == 3)) {
        snprintf(err, errlen, "D must be 2 or 3 (got %d)", D);
        return ESBGK_EINVAL;
    }
    if (!std::isfinite(tau) || !(tau > 0.5)) {
        snprintf(err, errlen, "tau must be > 1/2 (got %g)", tau);
        return ESBGK_EINVAL;
    }
    if (!std::isfinite(Pr) || !(Pr > 0)) {
        snprintf(err, errlen, "Pr must be > 0 (got %g)", Pr);
        return ESBGK_EINVAL;
    }
    if (Nf < 0 || Nf > 1000) {
        snprintf(err, errlen, "N_f must be in [0, 1000] (got %d)", Nf);
        return ESBGK_EINVAL;
    }
    if (!std::isfinite(kappa) || !(kappa >= 0 && kappa < 1)) {
        snprintf(err, errlen, "kappa must be in [0, 1) (got %g)", kappa);
        return ESBGK_EINVAL;
    }
    // stress rate 1/tau, heat-flux rate omega: (1/omega_s - 1/2)/(1/omega - 1/2) = Pr
    const double omega_s = 1.0 / tau;
    const double omega = 1.0 / (0.5 + (tau - 0.5) / Pr);
    const double nu = (1.0 - omega_s / omega) / (1.0 - kappa);
    // Lambda = (1-kappa)[(1-nu) T_tr delta + nu sigma] + kappa T_eq delta stays
    // positive definite for every sigma >= 0 with trace D T_tr (T_eq ~ T_tr).
    const double worst = nu >= 0 ? (1 - kappa) * (1 - nu) + kappa : (1 - kappa) * (1 + nu * (D - 1)) + kappa;
    if (!(worst > 0)) {
        snprintf(err, errlen, "Pr = %g, tau = %g, kappa = %g give nu = %g: Lambda can lose positive-definiteness",
                 Pr, tau, kappa, nu);
        return ESBGK_EINVAL;
    }
    out[0] = omega;
    out[1] = omega_s;
    out[2] = nu;
    out[3] = double(Nf + D + 2) / double(Nf + D);
    return ESBGK_OK;
}

}  // namespace esbgk

// L-BFGS-B, the bound-constrained quasi-Newton method the paper's PSF fits use:
// host-side iteration control in FP64 by reverse communication (the caller
// evaluates the loss and gradient wherever asked, here on the device).
//
// Each iteration (Byrd, Lu, Nocedal & Zhu 1995, with the projected subspace step
// of Morales & Nocedal 2011):
//  1. the generalized Cauchy point: the first local minimiser of the quadratic
//     model along the projected steepest-descent path, found by walking its
//     breakpoints in increasing order;
//  2. subspace minimisation of the model over the variables free at that point
//     (direct primal method through the compact representation
//     B = theta I - W M W^T, W = [Y, theta S]), the result projected onto the box,
//     or cut back to the box along the step when the projection is not a descent
//     direction;
//  3. a line search with the Moré-Thuente safeguarded cubic steps (sufficient
//     decrease 1e-3, curvature 0.9), from step 1 (1/|d| on the first iteration of
//     a problem without finite bounds on every variable), capped at the largest step
//     that keeps every bounded variable feasible;
//  4. the correction pair (s, y) kept when s^T y is safely positive.
// Convergence: projected-gradient infinity norm <= pgtol, or a relative decrease
// of f below factr * machine epsilon.
#include "starred.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

int starred_set_error(int code, const char *msg);

namespace {

constexpr double kFtol = 1e-3, kGtol = 0.9, kXtol = 0.1, kBig = 1e10;

double dot(const double *a, const double *b, long long n)
{
    double s = 0.0;
    for (long long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

// Solve A x = b (k x k, row major) by Gaussian elimination with partial pivoting;
// false when singular.
bool solve_dense(std::vector<double> A, std::vector<double> &b, int k)
{
    for (int c = 0; c < k; ++c) {
        int piv = c;
        for (int r = c + 1; r < k; ++r)
            if (std::fabs(A[r * k + c]) > std::fabs(A[piv * k + c])) piv = r;
        if (A[piv * k + c] == 0.0) return false;
        if (piv != c) {
            for (int j = 0; j < k; ++j) std::swap(A[c * k + j], A[piv * k + j]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < k; ++r) {
            const double f = A[r * k + c] / A[c * k + c];
            if (f == 0.0) continue;
            for (int j = c; j < k; ++j) A[r * k + j] -= f * A[c * k + j];
            b[r] -= f * b[c];
        }
    }
    for (int c = k - 1; c >= 0; --c) {
        double s = b[c];
        for (int j = c + 1; j < k; ++j) s -= A[c * k + j] * b[j];
        b[c] = s / A[c * k + c];
    }
    return true;
}

// Moré-Thuente: one safeguarded step of the interval [stx, sty] with the trial
// stp (function values f*, derivatives d*); updates the interval and the step.
void mt_step(double &stx, double &fx, double &dx, double &sty, double &fy, double &dy, double &stp, double fp,
             double dp, bool &brackt, double stpmin, double stpmax)
{
    const double sgnd = dp * (dx / std::fabs(dx));
    double stpf;
    if (fp > fx) {
        // higher value: the minimum is bracketed; cubic or the quadratic through fx, dx, fp
        const double theta = 3.0 * (fx - fp) / (stp - stx) + dx + dp;
        const double s = std::max(std::fabs(theta), std::max(std::fabs(dx), std::fabs(dp)));
        double gamma = s * std::sqrt((theta / s) * (theta / s) - (dx / s) * (dp / s));
        if (stp < stx) gamma = -gamma;
        const double p = (gamma - dx) + theta, q = ((gamma - dx) + gamma) + dp;
        const double stpc = stx + (p / q) * (stp - stx);
        const double stpq = stx + ((dx / ((fx - fp) / (stp - stx) + dx)) / 2.0) * (stp - stx);
        stpf = std::fabs(stpc - stx) < std::fabs(stpq - stx) ? stpc : stpc + (stpq - stpc) / 2.0;
        brackt = true;
    } else if (sgnd < 0.0) {
        // derivatives of opposite sign: bracketed; cubic or secant
        const double theta = 3.0 * (fx - fp) / (stp - stx) + dx + dp;
        const double s = std::max(std::fabs(theta), std::max(std::fabs(dx), std::fabs(dp)));
        double gamma = s * std::sqrt((theta / s) * (theta / s) - (dx / s) * (dp / s));
        if (stp > stx) gamma = -gamma;
        const double p = (gamma - dp) + theta, q = ((gamma - dp) + gamma) + dx;
        const double stpc = stp + (p / q) * (stx - stp);
        const double stpq = stp + (dp / (dp - dx)) * (stx - stp);
        stpf = std::fabs(stpc - stp) > std::fabs(stpq - stp) ? stpc : stpq;
        brackt = true;
    } else if (std::fabs(dp) < std::fabs(dx)) {
        // same sign, the derivative shrinks: cubic (if it points the right way) or secant
        const double theta = 3.0 * (fx - fp) / (stp - stx) + dx + dp;
        const double s = std::max(std::fabs(theta), std::max(std::fabs(dx), std::fabs(dp)));
        double gamma = s * std::sqrt(std::max(0.0, (theta / s) * (theta / s) - (dx / s) * (dp / s)));
        if (stp > stx) gamma = -gamma;
        const double p = (gamma - dp) + theta, q = (gamma + (dx - dp)) + gamma;
        const double r = p / q;
        double stpc;
        if (r < 0.0 && gamma != 0.0) stpc = stp + r * (stx - stp);
        else stpc = stp > stx ? stpmax : stpmin;
        const double stpq = stp + (dp / (dp - dx)) * (stx - stp);
        if (brackt) {
            stpf = std::fabs(stpc - stp) < std::fabs(stpq - stp) ? stpc : stpq;
            stpf = stp > stx ? std::min(stp + 0.66 * (sty - stp), stpf) : std::max(stp + 0.66 * (sty - stp), stpf);
        } else {
            stpf = std::fabs(stpc - stp) > std::fabs(stpq - stp) ? stpc : stpq;
            stpf = std::max(stpmin, std::min(stpmax, stpf));
        }
    } else {
        // same sign, the derivative does not shrink: cubic towards sty, or the far end
        if (brackt) {
            const double theta = 3.0 * (fp - fy) / (sty - stp) + dy + dp;
            const double s = std::max(std::fabs(theta), std::max(std::fabs(dy), std::fabs(dp)));
            double gamma = s * std::sqrt((theta / s) * (theta / s) - (dy / s) * (dp / s));
            if (stp > sty) gamma = -gamma;
            const double p = (gamma - dp) + theta, q = ((gamma - dp) + gamma) + dy;
            stpf = stp + (p / q) * (sty - stp);
        } else {
            stpf = stp > stx ? stpmax : stpmin;
        }
    }
    if (fp > fx) {
        sty = stp;
        fy = fp;
        dy = dp;
    } else {
        if (sgnd < 0.0) {
            sty = stx;
            fy = fx;
            dy = dx;
        }
        stx = stp;
        fx = fp;
        dx = dp;
    }
    stp = stpf;
}

// Moré-Thuente line search state (strong Wolfe conditions on phi(stp) = f(x + stp d)).
struct MoreThuente {
    enum { FG, CONV, WARN };
    bool brackt = false;
    int stage = 1;
    double finit = 0, ginit = 0, gtest = 0, width = 0, width1 = 0;
    double stx = 0, fx = 0, gx = 0, sty = 0, fy = 0, gy = 0, stmin = 0, stmax = 0;
    double stpmin = 0, stpmax = 0;

    // start at step stp with phi(0) = f, phi'(0) = g (< 0); the first trial is stp itself
    void start(double f, double g, double stp, double smin, double smax)
    {
        brackt = false;
        stage = 1;
        finit = f;
        ginit = g;
        gtest = kFtol * ginit;
        stpmin = smin;
        stpmax = smax;
        width = smax - smin;
        width1 = width / 0.5;
        stx = 0.0;
        fx = finit;
        gx = ginit;
        sty = 0.0;
        fy = finit;
        gy = ginit;
        stmin = 0.0;
        stmax = stp + 4.0 * stp;
    }
    // phi(stp) = f, phi'(stp) = g: CONV (accept stp), WARN (stop at stp), or FG with a new stp
    int next(double f, double g, double &stp)
    {
        const double ftest = finit + stp * gtest;
        if (stage == 1 && f <= ftest && g >= 0.0) stage = 2;
        if (brackt && (stp <= stmin || stp >= stmax)) return WARN;
        if (brackt && stmax - stmin <= kXtol * stmax) return WARN;
        if (stp == stpmax && f <= ftest && g <= gtest) return WARN;
        if (stp == stpmin && (f > ftest || g >= gtest)) return WARN;
        if (f <= ftest && std::fabs(g) <= kGtol * (-ginit)) return CONV;
        if (stage == 1 && f <= fx && f > ftest) {
            // the modified function psi(stp) = phi(stp) - phi(0) - gtest stp
            double fm = f - stp * gtest, fxm = fx - stx * gtest, fym = fy - sty * gtest;
            double gm = g - gtest, gxm = gx - gtest, gym = gy - gtest;
            mt_step(stx, fxm, gxm, sty, fym, gym, stp, fm, gm, brackt, stmin, stmax);
            fx = fxm + stx * gtest;
            fy = fym + sty * gtest;
            gx = gxm + gtest;
            gy = gym + gtest;
        } else {
            mt_step(stx, fx, gx, sty, fy, gy, stp, f, g, brackt, stmin, stmax);
        }
        if (brackt) {
            if (std::fabs(sty - stx) >= 0.66 * width1) stp = stx + 0.5 * (sty - stx);
            width1 = width;
            width = std::fabs(sty - stx);
            stmin = std::min(stx, sty);
            stmax = std::max(stx, sty);
        } else {
            stmin = stp + 1.1 * (stp - stx);
            stmax = stp + 4.0 * (stp - stx);
        }
        stp = std::max(stp, stpmin);
        stp = std::min(stp, stpmax);
        if ((brackt && (stp <= stmin || stp >= stmax)) || (brackt && stmax - stmin <= kXtol * stmax)) stp = stx;
        return FG;
    }
};

}  // namespace

struct starred_lbfgsb {
    long long n = 0;
    int m = 0, maxls = 20;
    double factr = 1e7, pgtol = 1e-5;
    std::vector<double> lo, hi;
    std::vector<char> haslo, hashi;
    bool constrained = false, boxed = true;
    // corrections, oldest first
    std::deque<std::vector<double>> S, Y;
    double theta = 1.0;
    std::vector<double> Mmat;  // the 2k x 2k middle matrix of the compact form (k = S.size())
    // iterate
    std::vector<double> x, g, xold, gold, d, z;
    double f = 0.0, fold = 0.0, gdold = 0.0, stp = 0.0;
    int iter = 0, nls = 0, state = 0, nfg = 0;
    MoreThuente ls;

    enum { ST_START, ST_FIRST, ST_LS };

    double proj_grad_norm() const
    {
        double s = 0.0;
        for (long long i = 0; i < n; ++i) {
            double gi = g[i];
            if (gi < 0.0) {
                if (hashi[i]) gi = std::max(x[i] - hi[i], gi);
            } else {
                if (haslo[i]) gi = std::min(x[i] - lo[i], gi);
            }
            s = std::max(s, std::fabs(gi));
        }
        return s;
    }
    // W^T v: [Y^T v ; theta S^T v]
    void wt(const double *v, std::vector<double> &out) const
    {
        const int k = (int)S.size();
        out.assign(2 * k, 0.0);
        for (int j = 0; j < k; ++j) {
            out[j] = dot(Y[j].data(), v, n);
            out[k + j] = theta * dot(S[j].data(), v, n);
        }
    }
    // row i of W: (y_1(i), .., y_k(i), theta s_1(i), ..)
    void wrow(long long i, std::vector<double> &out) const
    {
        const int k = (int)S.size();
        out.resize(2 * k);
        for (int j = 0; j < k; ++j) {
            out[j] = Y[j][i];
            out[k + j] = theta * S[j][i];
        }
    }
    void mmul(const std::vector<double> &v, std::vector<double> &out) const
    {
        const int k2 = (int)v.size();
        out.assign(k2, 0.0);
        for (int r = 0; r < k2; ++r) {
            double s = 0.0;
            for (int c = 0; c < k2; ++c) s += Mmat[(size_t)r * k2 + c] * v[c];
            out[r] = s;
        }
    }
    // M = [[-D, L^T], [L, theta S^T S]]^-1, L_ij = s_i^T y_j (i > j), D = diag(s_i^T y_i)
    bool form_m()
    {
        const int k = (int)S.size(), k2 = 2 * k;
        std::vector<double> A((size_t)k2 * k2, 0.0);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                const double sy = dot(S[i].data(), Y[j].data(), n);
                if (i == j) A[(size_t)i * k2 + j] = -sy;
                if (i > j) {
                    A[(size_t)(k + i) * k2 + j] = sy;  // L
                    A[(size_t)j * k2 + (k + i)] = sy;  // L^T
                }
                A[(size_t)(k + i) * k2 + (k + j)] = theta * dot(S[i].data(), S[j].data(), n);
            }
        Mmat.assign((size_t)k2 * k2, 0.0);
        for (int c = 0; c < k2; ++c) {
            std::vector<double> e(k2, 0.0);
            e[c] = 1.0;
            if (!solve_dense(A, e, k2)) return false;
            for (int r = 0; r < k2; ++r) Mmat[(size_t)r * k2 + c] = e[r];
        }
        return true;
    }

    // Generalized Cauchy point from x along -g: z and c = W^T (z - x).
    void cauchy(std::vector<double> &c)
    {
        const int k2 = 2 * (int)S.size();
        z = x;
        std::vector<double> dvec(n, 0.0), tb(n, kBig * kBig);
        std::vector<long long> brk;
        bool bounded_path = true;  // every moving variable meets a bound somewhere
        for (long long i = 0; i < n; ++i) {
            const double gi = g[i];
            double t = HUGE_VAL;
            if (gi < 0.0 && hashi[i]) t = (x[i] - hi[i]) / gi;
            else if (gi > 0.0 && haslo[i]) t = (x[i] - lo[i]) / gi;
            if (t == 0.0) continue;  // at a bound the gradient pushes against: fixed
            dvec[i] = -gi;
            if (t < HUGE_VAL) {
                tb[i] = t;
                brk.push_back(i);
            } else if (gi != 0.0) {
                bounded_path = false;
            }
        }
        std::sort(brk.begin(), brk.end(), [&](long long a, long long b) { return tb[a] < tb[b] || (tb[a] == tb[b] && a < b); });
        std::vector<double> p, tmp, wb, Mp, Mc, Mw;
        wt(dvec.data(), p);
        c.assign(k2, 0.0);
        double fp = -dot(dvec.data(), dvec.data(), n);  // g^T d
        double fpp = -theta * fp;
        if (k2) {
            mmul(p, Mp);
            fpp -= dot(p.data(), Mp.data(), k2);
        }
        if (fp >= 0.0) return;  // projected gradient is zero: z = x
        const double fpp0 = fpp;
        double dtm = -fp / fpp, told = 0.0;
        size_t ib = 0;
        while (ib < brk.size()) {
            const long long b = brk[ib];
            const double tj = tb[b], dt = tj - told;
            if (dtm < dt) break;
            // pass breakpoint b: variable b lands on its bound
            const double gb = g[b];
            const double zb_new = dvec[b] > 0.0 ? hi[b] : lo[b];
            const double zb = zb_new - x[b];
            z[b] = zb_new;
            for (int j = 0; j < k2; ++j) c[j] += dt * p[j];
            double wMc = 0.0, wMp = 0.0, wMw = 0.0;
            if (k2) {
                wrow(b, wb);
                mmul(c, Mc);
                mmul(p, Mp);
                mmul(wb, Mw);
                wMc = dot(wb.data(), Mc.data(), k2);
                wMp = dot(wb.data(), Mp.data(), k2);
                wMw = dot(wb.data(), Mw.data(), k2);
            }
            fp += dt * fpp + gb * gb + theta * gb * zb - gb * wMc;
            fpp -= theta * gb * gb + 2.0 * gb * wMp + gb * gb * wMw;
            fpp = std::max(DBL_EPSILON * fpp0, fpp);  // keeps the curvature positive
            for (int j = 0; j < k2; ++j) p[j] += gb * wb[j];
            dvec[b] = 0.0;
            told = tj;
            ++ib;
            if (ib == brk.size() && bounded_path) {
                dtm = 0.0;  // every moving variable has reached its bound
                break;
            }
            dtm = -fp / fpp;
        }
        dtm = std::max(dtm, 0.0);
        const double tt = told + dtm;
        for (long long i = 0; i < n; ++i)
            if (dvec[i] != 0.0) z[i] = x[i] + tt * dvec[i];
        for (int j = 0; j < k2; ++j) c[j] += dtm * p[j];
    }

    // Subspace minimisation over the variables free at z (direct primal method).
    void subspace(const std::vector<double> &c)
    {
        const int k = (int)S.size(), k2 = 2 * k;
        std::vector<long long> fr;
        for (long long i = 0; i < n; ++i) {
            const bool atlo = haslo[i] && z[i] <= lo[i], athi = hashi[i] && z[i] >= hi[i];
            if (!atlo && !athi) fr.push_back(i);
        }
        if (fr.empty() || k == 0) return;
        // reduced gradient r = Z^T (g + theta (z - x) - W M c)
        std::vector<double> Mc;
        mmul(c, Mc);
        std::vector<double> r(fr.size()), wrow_i;
        for (size_t q = 0; q < fr.size(); ++q) {
            const long long i = fr[q];
            wrow(i, wrow_i);
            r[q] = g[i] + theta * (z[i] - x[i]) - dot(wrow_i.data(), Mc.data(), k2);
        }
        // v = M W_Z^T r ; N = I - (1/theta) M W_Z^T W_Z ; v <- N^-1 v
        std::vector<double> wzr(k2, 0.0), WtW((size_t)k2 * k2, 0.0);
        for (size_t q = 0; q < fr.size(); ++q) {
            wrow(fr[q], wrow_i);
            for (int a = 0; a < k2; ++a) {
                wzr[a] += wrow_i[a] * r[q];
                for (int b = 0; b < k2; ++b) WtW[(size_t)a * k2 + b] += wrow_i[a] * wrow_i[b];
            }
        }
        std::vector<double> v;
        mmul(wzr, v);
        std::vector<double> Nm((size_t)k2 * k2, 0.0);
        for (int a = 0; a < k2; ++a)
            for (int b = 0; b < k2; ++b) {
                double s = 0.0;
                for (int e = 0; e < k2; ++e) s += Mmat[(size_t)a * k2 + e] * WtW[(size_t)e * k2 + b];
                Nm[(size_t)a * k2 + b] = (a == b ? 1.0 : 0.0) - s / theta;
            }
        if (!solve_dense(Nm, v, k2)) return;  // keep the Cauchy point
        // du = -(1/theta) r - (1/theta^2) W_Z v
        std::vector<double> du(fr.size());
        for (size_t q = 0; q < fr.size(); ++q) {
            wrow(fr[q], wrow_i);
            du[q] = -r[q] / theta - dot(wrow_i.data(), v.data(), k2) / (theta * theta);
        }
        // projection of z + du onto the box; kept if it is a descent direction from x
        std::vector<double> zp = z;
        for (size_t q = 0; q < fr.size(); ++q) {
            const long long i = fr[q];
            double t = z[i] + du[q];
            if (haslo[i]) t = std::max(lo[i], t);
            if (hashi[i]) t = std::min(hi[i], t);
            zp[i] = t;
        }
        double ddp = 0.0;
        for (long long i = 0; i < n; ++i) ddp += (zp[i] - x[i]) * g[i];
        if (ddp <= 0.0) {
            z.swap(zp);
            return;
        }
        // else the largest step along du from z that stays in the box (at most 1)
        double alpha = 1.0;
        long long ibd = -1;
        for (size_t q = 0; q < fr.size(); ++q) {
            const long long i = fr[q];
            const double dk = du[q];
            double t1 = alpha;
            if (dk < 0.0 && haslo[i]) {
                const double t2 = lo[i] - z[i];
                if (t2 >= 0.0) t1 = 0.0;
                else if (dk * alpha < t2) t1 = t2 / dk;
            } else if (dk > 0.0 && hashi[i]) {
                const double t2 = hi[i] - z[i];
                if (t2 <= 0.0) t1 = 0.0;
                else if (dk * alpha > t2) t1 = t2 / dk;
            }
            if (t1 < alpha) {
                alpha = t1;
                ibd = (long long)q;
            }
        }
        if (alpha < 1.0 && ibd >= 0) {
            const long long i = fr[ibd];
            if (du[ibd] > 0.0) z[i] = hi[i];
            else if (du[ibd] < 0.0) z[i] = lo[i];
            du[ibd] = 0.0;
        }
        for (size_t q = 0; q < fr.size(); ++q) z[fr[q]] += alpha * du[q];
    }

    // Direction and first trial step of an iteration; false when no descent is possible.
    bool begin_iteration()
    {
        std::vector<double> c;
        if (!constrained && !S.empty()) {
            z = x;
            c.assign(2 * S.size(), 0.0);
        } else {
            cauchy(c);
        }
        subspace(c);
        d.resize(n);
        for (long long i = 0; i < n; ++i) d[i] = z[i] - x[i];
        const double gd = dot(g.data(), d.data(), n);
        if (!(gd < 0.0)) return false;
        const double dnorm = std::sqrt(dot(d.data(), d.data(), n));
        // the largest step keeping every bounded variable feasible (1 on the first iteration)
        double stpmx = kBig;
        if (constrained) {
            if (iter == 0) {
                stpmx = 1.0;
            } else {
                for (long long i = 0; i < n; ++i) {
                    const double a1 = d[i];
                    if (a1 < 0.0 && haslo[i]) {
                        const double a2 = lo[i] - x[i];
                        if (a2 >= 0.0) stpmx = 0.0;
                        else if (a1 * stpmx < a2) stpmx = a2 / a1;
                    } else if (a1 > 0.0 && hashi[i]) {
                        const double a2 = hi[i] - x[i];
                        if (a2 <= 0.0) stpmx = 0.0;
                        else if (a1 * stpmx > a2) stpmx = a2 / a1;
                    }
                }
            }
        }
        stp = (iter == 0 && !boxed) ? std::min(1.0 / dnorm, stpmx) : 1.0;
        xold = x;
        gold = g;
        fold = f;
        gdold = gd;
        nls = 0;
        ls.start(f, gd, stp, 0.0, stpmx);
        for (long long i = 0; i < n; ++i) x[i] = xold[i] + stp * d[i];
        return true;
    }

    void restart_memory()
    {
        S.clear();
        Y.clear();
        theta = 1.0;
        Mmat.clear();
    }
};

extern "C" {

int starred_lbfgsb_create(int64_t n, int32_t m, const double *lo, const double *hi, double factr, double pgtol,
                          int32_t maxls, starred_lbfgsb **out)
{
    if (!out) return starred_set_error(STARRED_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || m < 1 || maxls < 1 || !(factr >= 0.0) || !(pgtol >= 0.0))
        return starred_set_error(STARRED_EINVAL, "n, m and maxls must be >= 1, factr and pgtol >= 0");
    starred_lbfgsb *s = new starred_lbfgsb();
    s->n = n;
    s->m = m;
    s->factr = factr;
    s->pgtol = pgtol;
    s->maxls = maxls;
    s->lo.assign(n, -HUGE_VAL);
    s->hi.assign(n, HUGE_VAL);
    s->haslo.assign(n, 0);
    s->hashi.assign(n, 0);
    for (long long i = 0; i < n; ++i) {
        if (lo && std::isfinite(lo[i])) {
            s->lo[i] = lo[i];
            s->haslo[i] = 1;
        }
        if (hi && std::isfinite(hi[i])) {
            s->hi[i] = hi[i];
            s->hashi[i] = 1;
        }
        if (s->haslo[i] && s->hashi[i] && s->lo[i] > s->hi[i]) {
            delete s;
            return starred_set_error(STARRED_EINVAL, "lower bound above upper bound");
        }
        s->constrained = s->constrained || s->haslo[i] || s->hashi[i];
        s->boxed = s->boxed && s->haslo[i] && s->hashi[i];
    }
    *out = s;
    return STARRED_OK;
}

int starred_lbfgsb_destroy(starred_lbfgsb *s)
{
    if (!s) return starred_set_error(STARRED_EINVAL, "state is NULL");
    delete s;
    return STARRED_OK;
}

int starred_lbfgsb_iterate(starred_lbfgsb *s, double *x, double f, const double *g, int32_t *task)
{
    if (!s || !x || !task) return starred_set_error(STARRED_EINVAL, "NULL argument");
    const long long n = s->n;
    if (s->state == starred_lbfgsb::ST_START) {
        s->x.assign(x, x + n);
        for (long long i = 0; i < n; ++i) {
            if (s->haslo[i]) s->x[i] = std::max(s->x[i], s->lo[i]);
            if (s->hashi[i]) s->x[i] = std::min(s->x[i], s->hi[i]);
        }
        std::copy(s->x.begin(), s->x.end(), x);
        s->state = starred_lbfgsb::ST_FIRST;
        *task = STARRED_LBFGSB_FG;
        return STARRED_OK;
    }
    if (!g) return starred_set_error(STARRED_EINVAL, "g is NULL");
    ++s->nfg;
    if (s->state == starred_lbfgsb::ST_FIRST) {
        s->f = f;
        s->g.assign(g, g + n);
        if (s->proj_grad_norm() <= s->pgtol) {
            *task = STARRED_LBFGSB_CONVERGED;
            return STARRED_OK;
        }
        if (!s->begin_iteration()) {
            *task = STARRED_LBFGSB_ABNORMAL;
            return STARRED_OK;
        }
        std::copy(s->x.begin(), s->x.end(), x);
        s->state = starred_lbfgsb::ST_LS;
        *task = STARRED_LBFGSB_FG;
        return STARRED_OK;
    }
    // line search: (f, g) at x = xold + stp d
    s->f = f;
    s->g.assign(g, g + n);
    const double gd = dot(s->g.data(), s->d.data(), n);
    ++s->nls;
    double stp = s->stp;
    const int r = s->ls.next(f, gd, stp);
    if (r == MoreThuente::FG && s->nls < s->maxls && stp != s->stp) {
        s->stp = stp;
        for (long long i = 0; i < n; ++i) s->x[i] = s->xold[i] + stp * s->d[i];
        std::copy(s->x.begin(), s->x.end(), x);
        *task = STARRED_LBFGSB_FG;
        return STARRED_OK;
    }
    if (r == MoreThuente::FG) {
        // too many trials: back to the last iterate; with history, forget it and retry
        s->x = s->xold;
        s->g = s->gold;
        s->f = s->fold;
        std::copy(s->x.begin(), s->x.end(), x);
        if (s->S.empty()) {
            *task = STARRED_LBFGSB_ABNORMAL;
            return STARRED_OK;
        }
        s->restart_memory();
        if (!s->begin_iteration()) {
            *task = STARRED_LBFGSB_ABNORMAL;
            return STARRED_OK;
        }
        std::copy(s->x.begin(), s->x.end(), x);
        *task = STARRED_LBFGSB_FG;
        return STARRED_OK;
    }
    // the step is accepted: an iteration ends at x
    ++s->iter;
    // correction pair s = stp d, y = g - gold
    {
        const double dr = (gd - s->gdold) * s->stp;
        const double ddum = -s->gdold * s->stp;
        if (dr > DBL_EPSILON * ddum) {
            std::vector<double> sv(n), yv(n);
            for (long long i = 0; i < n; ++i) {
                sv[i] = s->stp * s->d[i];
                yv[i] = s->g[i] - s->gold[i];
            }
            const double rr = dot(yv.data(), yv.data(), n);
            if ((int)s->S.size() == s->m) {
                s->S.pop_front();
                s->Y.pop_front();
            }
            s->S.push_back(std::move(sv));
            s->Y.push_back(std::move(yv));
            s->theta = rr / dr;
            if (!s->form_m()) s->restart_memory();
        }
    }
    const double sbg = s->proj_grad_norm();
    const double ddum = std::max(std::fabs(s->fold), std::max(std::fabs(s->f), 1.0));
    if (sbg <= s->pgtol || s->fold - s->f <= s->factr * DBL_EPSILON * ddum) {
        s->state = starred_lbfgsb::ST_FIRST;  // a further call restarts from here
        --s->nfg;                             // (that call re-supplies f, g at x)
        *task = STARRED_LBFGSB_CONVERGED;
        return STARRED_OK;
    }
    // the next iteration's first trial, announced as NEW_X with x unchanged: the
    // caller continues by passing the same (f, g) back
    s->state = starred_lbfgsb::ST_FIRST;
    --s->nfg;
    *task = STARRED_LBFGSB_NEW_X;
    return STARRED_OK;
}

int starred_lbfgsb_counts(const starred_lbfgsb *s, int32_t *iterations, int32_t *evaluations)
{
    if (!s) return starred_set_error(STARRED_EINVAL, "state is NULL");
    if (iterations) *iterations = s->iter;
    if (evaluations) *evaluations = s->nfg;
    return STARRED_OK;
}

}  // extern "C"

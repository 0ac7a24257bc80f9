/*
 * Oracle for the spin Hamiltonian, the LLG equation and the Heun scheme.
 * TEST INFRASTRUCTURE ONLY (see sllg_oracle.h).
 *
 * Paper passages followed (Evans et al., arXiv:1310.6143):
 *  - "The classical spin Hamiltonian": exchange -sum_{i!=j} J_ij S_i.S_j,
 *    uniaxial anisotropy -k_u sum_i (S_i.e)^2, applied field
 *    -sum_i mu_s S_i.H_app.  J is given in joules per link (Table 1), so
 *    each link enters the energy once and the field on spin i from
 *    neighbour j is J_ij S_j / mu_s.  Tensorial exchange replaces the
 *    scalar by a 3x3 matrix, energy -S_i^T J_ij S_j per link; with
 *    J_ji = J_ij^T the field on i is again (1/mu_s) sum_j J_ij S_j (matrix
 *    times vector).  Cubic anisotropy (k_c/2)(Sx^4 + Sy^4 + Sz^4) per site
 *    gives the field -(2 k_c/mu_s)(Sx^3, Sy^3, Sz^3).
 *  - "Spin Dynamics": the atomistic LLG equation and the effective field
 *    H_i = -(1/mu_s) dH/dS_i.
 *  - "Langevin Dynamics": the thermal field Gamma sqrt(2 lambda kB T /
 *    (gamma mu_s dt)), added to the effective field.
 *  - "Demagnetising fields": the macrocell field (demag.c), added to the
 *    effective field of every atom of a cell, held fixed between updates.
 *  - "Time Integration of the LLG Equation": Heun predictor on every spin,
 *    renormalisation, field re-evaluated at the predicted spins with the
 *    same thermal field, corrector from the original spin with the mean of
 *    the two slopes, renormalisation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "sllg_oracle.h"

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Scale v to unit length; -1 if its length is zero or not finite. */
static int normalise3(double v[3])
{
    double len = sqrt(dot3(v, v));
    if (!(len > 0.0) || !isfinite(len))
        return -1;
    v[0] /= len;
    v[1] /= len;
    v[2] /= len;
    return 0;
}

/* Exchange field of spin i: (1/mu_s,i) sum over the links of row i of
 * J[type] S_j, the negative derivative of -sum_{i!=j} J_ij S_i.S_j; with
 * tensors, the matrix J_tensor[type] applied to S_j. */
void orc_exchange_field(const orc_system *s, const double *S, int64_t i, double h[3])
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t k = s->row_ptr[i]; k < s->row_ptr[i + 1]; ++k) {
        int64_t j = s->col[k];
        const int t = s->ntype ? s->ntype[k] : 0;
        const double *sj = S + 3 * j;
        if (s->J_tensor) {
            const double *M = s->J_tensor + 9 * t;
            for (int a = 0; a < 3; ++a)
                acc[a] += M[3 * a + 0] * sj[0] + M[3 * a + 1] * sj[1] + M[3 * a + 2] * sj[2];
        } else {
            double Jij = s->J[t];
            acc[0] += Jij * sj[0];
            acc[1] += Jij * sj[1];
            acc[2] += Jij * sj[2];
        }
    }
    h[0] = acc[0] / s->mu_s[i];
    h[1] = acc[1] / s->mu_s[i];
    h[2] = acc[2] / s->mu_s[i];
}

/* Deterministic effective field: exchange + uniaxial anisotropy
 * (2 k_u / mu_s)(S.e) e + applied field (+ cubic anisotropy). */
void orc_effective_field(const orc_system *s, const double *S, int64_t i, double h[3])
{
    const double *e = s->easy_axis + 3 * i;
    const double *si = S + 3 * i;
    orc_exchange_field(s, S, i, h);
    double a = 2.0 * s->k_u[i] / s->mu_s[i] * dot3(si, e);
    h[0] += a * e[0] + s->H[0];
    h[1] += a * e[1] + s->H[1];
    h[2] += a * e[2] + s->H[2];
    if (s->k_c) {
        /* -(1/mu_s) d/dS of (k_c/2) sum_a S_a^4 */
        const double c = -2.0 * s->k_c[i] / s->mu_s[i];
        for (int q = 0; q < 3; ++q)
            h[q] += c * si[q] * si[q] * si[q];
    }
    if (s->demag && s->demag->valid)
        for (int q = 0; q < 3; ++q)
            h[q] += s->demag->field[3 * i + q];
}

void orc_effective_fields(const orc_system *s, const double *S, double *H_out)
{
    for (int64_t i = 0; i < s->n; ++i)
        orc_effective_field(s, S, i, H_out + 3 * i);
}

/* dS/dt = -gamma/(1+lambda^2) [S x H + lambda S x (S x H)]. */
void orc_llg_rhs(double gamma, double alpha, const double spin[3], const double h[3], double ds[3])
{
    double sxh[3], sxsxh[3];
    cross3(spin, h, sxh);
    cross3(spin, sxh, sxsxh);
    double pre = -gamma / (1.0 + alpha * alpha);
    ds[0] = pre * (sxh[0] + alpha * sxsxh[0]);
    ds[1] = pre * (sxh[1] + alpha * sxsxh[1]);
    ds[2] = pre * (sxh[2] + alpha * sxsxh[2]);
}

/* Width of the thermal field, sqrt(2 lambda kB T / (gamma mu_s dt)). */
double orc_thermal_sigma(const orc_system *s, int64_t i)
{
    return sqrt(2.0 * s->alpha * ORC_KB * s->temperature / (s->gamma * s->mu_s[i] * s->dt));
}

double orc_energy(const orc_system *s, const double *S)
{
    double total = 0.0;
    for (int64_t i = 0; i < s->n; ++i) {
        const double *si = S + 3 * i;
        const double *e = s->easy_axis + 3 * i;
        double hex[3];
        orc_exchange_field(s, S, i, hex);
        double se = dot3(si, e);
        /* each link is listed in both rows, so half of mu_s S.H_exc per row */
        double exc = 0.5 * s->mu_s[i] * dot3(si, hex);
        double ani = s->k_u[i] * se * se;
        double app = s->mu_s[i] * dot3(si, s->H);
        total -= exc + ani + app;
        if (s->k_c) {
            const double x2 = si[0] * si[0], y2 = si[1] * si[1], z2 = si[2] * si[2];
            total += 0.5 * s->k_c[i] * (x2 * x2 + y2 * y2 + z2 * z2);
        }
    }
    return total;
}

void orc_magnetisation(const orc_system *s, const double *S, double m[3])
{
    double acc[3] = {0.0, 0.0, 0.0}, mu = 0.0;
    for (int64_t i = 0; i < s->n; ++i) {
        acc[0] += s->mu_s[i] * S[3 * i + 0];
        acc[1] += s->mu_s[i] * S[3 * i + 1];
        acc[2] += s->mu_s[i] * S[3 * i + 2];
        mu += s->mu_s[i];
    }
    m[0] = acc[0] / mu;
    m[1] = acc[1] / mu;
    m[2] = acc[2] / mu;
}

int orc_heun_step(const orc_system *s, double *S, uint64_t step, double *work)
{
    const int64_t n = s->n;
    double *Sp = work;          /* predicted spins S' */
    double *dS = work + 3 * n;  /* predictor slope */
    double *Hth = work + 6 * n; /* thermal field, fixed for the whole step */

    /* Demagnetising field: updated from the current spins on schedule,
     * then fixed for the whole step like the thermal field. */
    if (s->demag && (!s->demag->valid || step % (uint64_t)s->demag->every == 0))
        if (orc_demag_update(s, S))
            return -2;

    /* Thermal field of this step, one draw per spin. */
    for (int64_t i = 0; i < n; ++i) {
        double g[3];
        double sigma = orc_thermal_sigma(s, i);
        orc_gaussian3(s->seed, step, (uint64_t)i, 0u, g);
        Hth[3 * i + 0] = sigma * g[0];
        Hth[3 * i + 1] = sigma * g[1];
        Hth[3 * i + 2] = sigma * g[2];
    }

    /* Predictor on every spin: S' = S + dS dt, renormalised. */
    for (int64_t i = 0; i < n; ++i) {
        double h[3];
        orc_effective_field(s, S, i, h);
        h[0] += Hth[3 * i + 0];
        h[1] += Hth[3 * i + 1];
        h[2] += Hth[3 * i + 2];
        orc_llg_rhs(s->gamma, s->alpha, S + 3 * i, h, dS + 3 * i);
        for (int c = 0; c < 3; ++c)
            Sp[3 * i + c] = S[3 * i + c] + dS[3 * i + c] * s->dt;
        if (normalise3(Sp + 3 * i))
            return -1;
    }

    /* Corrector on every spin, from the original S with the mean slope. */
    for (int64_t i = 0; i < n; ++i) {
        double h[3], dSp[3];
        orc_effective_field(s, Sp, i, h);
        h[0] += Hth[3 * i + 0];
        h[1] += Hth[3 * i + 1];
        h[2] += Hth[3 * i + 2];
        orc_llg_rhs(s->gamma, s->alpha, Sp + 3 * i, h, dSp);
        for (int c = 0; c < 3; ++c)
            S[3 * i + c] = S[3 * i + c] + 0.5 * (dS[3 * i + c] + dSp[c]) * s->dt;
        if (normalise3(S + 3 * i))
            return -1;
    }
    return 0;
}

int orc_integrate(const orc_system *s, double *S, uint64_t step0, int64_t n_steps,
                  double *m_out, double *E_out)
{
    double *work = (double *)malloc(sizeof(double) * 9 * (size_t)(s->n > 0 ? s->n : 1));
    if (!work)
        return -2;
    int rc = 0;
    for (int64_t t = 0; t < n_steps; ++t) {
        const int st = orc_heun_step(s, S, step0 + (uint64_t)t, work);
        if (st) {
            rc = st;
            break;
        }
        if (m_out)
            orc_magnetisation(s, S, m_out + 3 * t);
        if (E_out)
            E_out[t] = orc_energy(s, S);
    }
    free(work);
    return rc;
}

double orc_max_torque(const orc_system *s, const double *S)
{
    double worst = 0.0;
    for (int64_t i = 0; i < s->n; ++i) {
        double h[3], t[3];
        orc_effective_field(s, S, i, h);
        cross3(S + 3 * i, h, t);
        double mag = sqrt(dot3(t, t));
        if (mag > worst)
            worst = mag;
    }
    return worst;
}

int64_t orc_relax(const orc_system *s, double *S, double torque_tol, int64_t max_steps,
                  uint64_t step0)
{
    double *work = (double *)malloc(sizeof(double) * 9 * (size_t)(s->n > 0 ? s->n : 1));
    if (!work)
        return -2;
    int64_t taken = 0;
    if (s->demag && !s->demag->valid && orc_demag_update(s, S)) {
        free(work);
        return -2;
    }
    while (orc_max_torque(s, S) > torque_tol) {
        if (taken >= max_steps) {
            free(work);
            return -1;
        }
        orc_heun_step(s, S, step0 + (uint64_t)taken, work);
        ++taken;
    }
    free(work);
    return taken;
}

int64_t orc_neighbours(int64_t n, const double *pos, const double box[3], int n_shells,
                       const double *shell_lo, const double *shell_hi,
                       int64_t *row_ptr, int32_t *col, uint8_t *ntype, int64_t cap)
{
    int64_t count = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double d[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = pos[3 * j + a] - pos[3 * i + a];
                if (box[a] > 0.0)
                    d[a] -= box[a] * nearbyint(d[a] / box[a]);
            }
            double r = sqrt(dot3(d, d));
            for (int t = 0; t < n_shells; ++t) {
                if (r >= shell_lo[t] && r <= shell_hi[t]) {
                    if (count >= cap)
                        return -1;
                    col[count] = (int32_t)j;
                    ntype[count] = (uint8_t)t;
                    ++count;
                    break;
                }
            }
        }
        row_ptr[i + 1] = count;
    }
    return count;
}

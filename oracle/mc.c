/*
 * Monte Carlo Metropolis sampling of the classical spin Hamiltonian with the
 * Hinzke-Nowak mixture of trial moves (section "Monte Carlo Methods").
 * TEST INFRASTRUCTURE ONLY (see sllg_oracle.h).
 *
 * A trial on spin i draws one of three moves with equal probability:
 * reversal S' = -S, a Gaussian move S' = |S + sigma_g Gamma| with the cone
 * width sigma_g = (2/25)(kB T/muB)^(1/5), or a uniform point on the sphere
 * S' = Gamma/|Gamma|.  It is accepted with probability exp(-dE/(kB T)),
 * unconditionally when dE <= 0.
 *
 * Two orders of the N trials of one Monte Carlo step:
 *
 * - the paper's (orc_mc_step_random): N trials, each on a site drawn
 *   uniformly at random with replacement.  Trial t of step k takes its
 *   site, move and acceptance uniform from Philox counter (t, k lo, k hi, 4)
 *   and its Gaussian numbers from counter (t, k lo, k hi, 5);
 * - colour classes (orc_mc_step): every site once, colour class by colour
 *   class of a greedy colouring of the neighbour graph (ascending colour,
 *   ascending site within a colour).  Sites of one colour share no link, so
 *   their trials do not interact and the order within a class is
 *   immaterial.  The greedy colouring visits the sites in ascending order,
 *   or (orc_mc_run_visit) in a given order: on a lattice, grouped by basis
 *   site and by the parity of the cell's x + y + z (orc_lattice_visit),
 *   which gives the bcc lattice with first and second neighbours four
 *   classes of N/4 sites where ascending order gives ten of very unequal
 *   size.  The Gaussian numbers of site i at step k come from counter
 *   (i, k lo, k hi, 2), the move choice and the acceptance uniform from
 *   counter (i, k lo, k hi, 3).
 *
 * Every single trial satisfies detailed balance, so both chains sample the
 * same Boltzmann distribution; the test suite checks that their averages
 * agree within their statistical errors.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "sllg_oracle.h"

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

int orc_greedy_colours_in(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *visit,
                          int32_t *colour)
{
    int n_colours = 0;
    for (int64_t i = 0; i < n; ++i)
        colour[i] = -1;   /* not coloured yet */
    /* a site has at most (row length) coloured neighbours, so a free colour
     * exists among the first (row length + 1) */
    for (int64_t v = 0; v < n; ++v) {
        const int64_t i = visit ? visit[v] : v;
        const int64_t deg = row_ptr[i + 1] - row_ptr[i];
        char *used = (char *)calloc((size_t)deg + 1, 1);
        if (!used)
            return -1;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int64_t j = col[k];
            if (colour[j] >= 0 && colour[j] <= deg)
                used[colour[j]] = 1;
        }
        int c = 0;
        while (used[c])
            ++c;
        free(used);
        colour[i] = c;
        if (c + 1 > n_colours)
            n_colours = c + 1;
    }
    return n_colours;
}

int orc_greedy_colours(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *colour)
{
    return orc_greedy_colours_in(n, row_ptr, col, NULL, colour);
}

int orc_lattice_visit(int64_t n, int nb, const int cells[3], int64_t *visit)
{
    if (nb < 1 || (int64_t)nb * cells[0] * cells[1] * cells[2] != n)
        return -1;
    /* site i = b + nb (x + cells[0] (y + cells[1] z)): the sites of basis
     * site 0 with x + y + z even, then odd, then basis site 1, ...; each
     * group in ascending site order */
    int64_t v = 0;
    for (int b = 0; b < nb; ++b)
        for (int parity = 0; parity < 2; ++parity)
            for (int64_t i = 0; i < n; ++i) {
                const int64_t cell = i / nb;
                const int64_t x = cell % cells[0], y = (cell / cells[0]) % cells[1],
                              z = cell / ((int64_t)cells[0] * cells[1]);
                if (i % nb == b && (x + y + z) % 2 == parity)
                    visit[v++] = i;
            }
    return 0;
}

double orc_mc_cone_width(double temperature)
{
    return 2.0 / 25.0 * pow(ORC_KB * temperature / ORC_MUB, 0.2);
}

void orc_mc_choice(uint64_t seed, uint64_t step, uint64_t site, uint32_t *move, double *u)
{
    const uint32_t ctr[4] = {(uint32_t)site, (uint32_t)step, (uint32_t)(step >> 32), 3u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    *move = (uint32_t)(((uint64_t)r[0] * 3u) >> 32);   /* 0, 1 or 2, each with probability 1/3 */
    *u = (double)r[1] * (1.0 / 4294967296.0);          /* uniform in [0, 1) */
}

/* Energy of spin i's terms when it points along x, with the neighbours as
 * they are: -x.(sum_j J_ij S_j) - k_u (x.e)^2 - mu_s x.H, plus
 * (k_c/2)(x_x^4 + x_y^4 + x_z^4) with cubic anisotropy; J_ij S_j is a
 * matrix product with tensorial exchange. */
static double site_energy(const orc_system *s, const double *S, int64_t i, const double x[3])
{
    double sum[3] = {0.0, 0.0, 0.0};
    for (int64_t k = s->row_ptr[i]; k < s->row_ptr[i + 1]; ++k) {
        const int t = s->ntype ? s->ntype[k] : 0;
        const double *sj = S + 3 * (int64_t)s->col[k];
        if (s->J_tensor) {
            const double *M = s->J_tensor + 9 * t;
            for (int a = 0; a < 3; ++a)
                sum[a] += M[3 * a + 0] * sj[0] + M[3 * a + 1] * sj[1] + M[3 * a + 2] * sj[2];
        } else {
            const double J = s->J[t];
            sum[0] += J * sj[0];
            sum[1] += J * sj[1];
            sum[2] += J * sj[2];
        }
    }
    const double xe = dot3(x, s->easy_axis + 3 * i);
    double E = -dot3(x, sum) - s->k_u[i] * xe * xe - s->mu_s[i] * dot3(x, s->H);
    if (s->k_c) {
        const double x2 = x[0] * x[0], y2 = x[1] * x[1], z2 = x[2] * x[2];
        E += 0.5 * s->k_c[i] * (x2 * x2 + y2 * y2 + z2 * z2);
    }
    return E;
}

/* One Metropolis trial on spin i with its random numbers given: move type,
 * acceptance uniform u and three Gaussian numbers g.  Returns 1 when
 * accepted. */
static int mc_trial_with(const orc_system *s, double *S, int64_t i, uint32_t move, double u, const double g[3])
{
    double *si = S + 3 * i;
    double trial[3];
    if (move == 0) {            /* spin flip */
        trial[0] = -si[0];
        trial[1] = -si[1];
        trial[2] = -si[2];
    } else {
        if (move == 1) {        /* Gaussian move in a cone around S */
            const double w = orc_mc_cone_width(s->temperature);
            for (int c = 0; c < 3; ++c)
                trial[c] = si[c] + w * g[c];
        } else {                /* uniform on the sphere */
            for (int c = 0; c < 3; ++c)
                trial[c] = g[c];
        }
        const double len = sqrt(dot3(trial, trial));
        if (!(len > 0.0))
            return 0;
        trial[0] /= len;
        trial[1] /= len;
        trial[2] /= len;
    }
    const double dE = site_energy(s, S, i, trial) - site_energy(s, S, i, si);
    int accept = dE <= 0.0;
    if (!accept && s->temperature > 0.0)
        accept = u < exp(-dE / (ORC_KB * s->temperature));
    if (accept) {
        si[0] = trial[0];
        si[1] = trial[1];
        si[2] = trial[2];
    }
    return accept;
}

int orc_mc_trial(const orc_system *s, double *S, int64_t i, uint64_t step)
{
    uint32_t move;
    double u, g[3];
    orc_mc_choice(s->seed, step, (uint64_t)i, &move, &u);
    orc_gaussian3(s->seed, step, (uint64_t)i, 2u, g);
    return mc_trial_with(s, S, i, move, u, g);
}

int64_t orc_mc_step_random(const orc_system *s, double *S, uint64_t step)
{
    const uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
    int64_t accepted = 0;
    for (int64_t t = 0; t < s->n; ++t) {
        const uint32_t ctr[4] = {(uint32_t)t, (uint32_t)step, (uint32_t)(step >> 32), 4u};
        uint32_t r[4];
        orc_philox4x32_10(ctr, key, r);
        /* site: a 64-bit uniform scaled to [0, n) */
        const uint64_t x = (uint64_t)r[0] | ((uint64_t)r[1] << 32);
        const int64_t i = (int64_t)(((unsigned __int128)x * (uint64_t)s->n) >> 64);
        const uint32_t move = (uint32_t)(((uint64_t)r[2] * 3u) >> 32);
        const double u = (double)r[3] * (1.0 / 4294967296.0);
        double g[3];
        orc_gaussian3(s->seed, step, (uint64_t)t, 5u, g);
        accepted += mc_trial_with(s, S, i, move, u, g);
    }
    return accepted;
}

int64_t orc_mc_step(const orc_system *s, double *S, const int32_t *colour, int n_colours, uint64_t step)
{
    int64_t accepted = 0;
    for (int c = 0; c < n_colours; ++c)
        for (int64_t i = 0; i < s->n; ++i)
            if (colour[i] == c)
                accepted += orc_mc_trial(s, S, i, step);
    return accepted;
}

int orc_mc_run(const orc_system *s, double *S, uint64_t step0, int64_t n_steps, double *m_out,
               double *E_out, int64_t *accepted_out)
{
    return orc_mc_run_visit(s, NULL, S, step0, n_steps, m_out, E_out, accepted_out);
}

int orc_mc_run_visit(const orc_system *s, const int64_t *visit, double *S, uint64_t step0, int64_t n_steps,
                     double *m_out, double *E_out, int64_t *accepted_out)
{
    int32_t *colour = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s->n > 0 ? s->n : 1));
    if (!colour)
        return -2;
    if (s->demag) {   /* not defined for Monte Carlo here */
        free(colour);
        return -3;
    }
    const int n_colours = orc_greedy_colours_in(s->n, s->row_ptr, s->col, visit, colour);
    if (n_colours < 0) {
        free(colour);
        return -2;
    }
    for (int64_t t = 0; t < n_steps; ++t) {
        const int64_t acc = orc_mc_step(s, S, colour, n_colours, step0 + (uint64_t)t);
        if (accepted_out)
            accepted_out[t] = acc;
        if (m_out)
            orc_magnetisation(s, S, m_out + 3 * t);
        if (E_out)
            E_out[t] = orc_energy(s, S);
    }
    free(colour);
    return 0;
}

int orc_mc_run_random(const orc_system *s, double *S, uint64_t step0, int64_t n_steps, double *m_out,
                      double *E_out, int64_t *accepted_out)
{
    if (s->demag)
        return -3;
    for (int64_t t = 0; t < n_steps; ++t) {
        const int64_t acc = orc_mc_step_random(s, S, step0 + (uint64_t)t);
        if (accepted_out)
            accepted_out[t] = acc;
        if (m_out)
            orc_magnetisation(s, S, m_out + 3 * t);
        if (E_out)
            E_out[t] = orc_energy(s, S);
    }
    return 0;
}

/*
 * Macrocell demagnetising field (section "Demagnetising fields").
 * TEST INFRASTRUCTURE ONLY (see sllg_oracle.h).
 *
 * The sample is cut into cubic macrocells of edge cell_size, the grid
 * starting a thousandth of a cell below the smallest atom coordinate along
 * each axis (cell index floor((x - x_min + cell_size/1000) / cell_size)), so
 * that atomic planes lying on a cell boundary fall into the upper cell
 * whatever the rounding of their coordinates; only cells holding atoms take
 * part.  For every cell p:
 *   - moment m_p = sum_i mu_s,i S_i over its atoms;
 *   - position: the magnetic centre of mass sum_i mu_s,i x_i / sum_i mu_s,i;
 *   - volume V_p = (atoms in the cell) * atom_volume (atom_volume = unit-cell
 *     volume / atoms per unit cell);
 *   - field H_p = mu0/(4 pi) sum_{q != p} [3 (m_q . r) r - m_q] / |x_q - x_p|^3
 *     - (mu0/3) m_p / V_p, r the unit vector from p to q (the dipole sum
 *     over the other cells plus the self field of a cube, demagnetising
 *     factor 1/3).
 * Every atom takes the field of its cell.  The printed pair matrix M_pq is
 * garbled; it is rederived from the dipole expression: M_pq =
 * (3 r r^T - I) / |x_q - x_p|^3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "sllg_oracle.h"

#define ORC_MU0_OVER_4PI 1e-7   /* T m / A, classical SI value of mu0/(4 pi) */
#define ORC_PI 3.14159265358979323846

typedef struct {
    int64_t key;
    int64_t site;
} keyed;

static int by_key(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return x->site < y->site ? -1 : (x->site > y->site);
}

/* Bins the atoms into macrocells: cell[i] (cells numbered in ascending
 * grid key) and per cell {atoms, sum mu, sum mu x (3), sum mu S (3)} in a
 * fresh array *acc_out of 8 * (*n_mc) doubles.  0, or -2 when out of memory. */
static int bin_cells(const orc_system *s, const double *S, int64_t *cell, double **acc_out, int64_t *n_mc_out)
{
    const orc_demag *d = s->demag;
    const int64_t n = s->n;
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a)
        lo[a] = hi[a] = d->pos[a];
    for (int64_t i = 1; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            const double x = d->pos[3 * i + a];
            lo[a] = x < lo[a] ? x : lo[a];
            hi[a] = x > hi[a] ? x : hi[a];
        }
    for (int a = 0; a < 3; ++a)
        lo[a] -= d->cell_size / 1000.0;
    int64_t dims[3];
    for (int a = 0; a < 3; ++a)
        dims[a] = (int64_t)floor((hi[a] - lo[a]) / d->cell_size) + 1;
    keyed *ks = (keyed *)malloc(sizeof(keyed) * (size_t)n);
    if (!ks)
        return -2;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a)
            c[a] = (int64_t)floor((d->pos[3 * i + a] - lo[a]) / d->cell_size);
        ks[i].key = (c[0] * dims[1] + c[1]) * dims[2] + c[2];
        ks[i].site = i;
    }
    qsort(ks, (size_t)n, sizeof(keyed), by_key);
    int64_t n_mc = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (k == 0 || ks[k].key != ks[k - 1].key)
            ++n_mc;
        cell[ks[k].site] = n_mc - 1;
    }
    free(ks);
    double *acc = (double *)calloc((size_t)n_mc * 8, sizeof(double));
    if (!acc)
        return -2;
    for (int64_t i = 0; i < n; ++i) {
        double *c = acc + 8 * cell[i];
        const double mu = s->mu_s[i];
        c[0] += 1.0;
        c[1] += mu;
        for (int a = 0; a < 3; ++a) {
            c[2 + a] += mu * d->pos[3 * i + a];
            c[5 + a] += mu * S[3 * i + a];
        }
    }
    *acc_out = acc;
    *n_mc_out = n_mc;
    return 0;
}

/* Field of cell p: the dipole sum over every other cell plus the self term. */
static void cell_field(const double *acc, int64_t n_mc, int64_t p, double atom_volume, double out[3])
{
    const double *cp = acc + 8 * p;
    double xp[3];
    for (int a = 0; a < 3; ++a)
        xp[a] = cp[2 + a] / cp[1];
    double h[3] = {0.0, 0.0, 0.0};
    for (int64_t q = 0; q < n_mc; ++q) {
        if (q == p)
            continue;
        const double *cq = acc + 8 * q;
        double r[3];
        for (int a = 0; a < 3; ++a)
            r[a] = cq[2 + a] / cq[1] - xp[a];
        const double dist = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int a = 0; a < 3; ++a)
            r[a] /= dist;
        const double *mq = cq + 5;
        const double mr = mq[0] * r[0] + mq[1] * r[1] + mq[2] * r[2];
        const double inv3 = 1.0 / (dist * dist * dist);
        for (int a = 0; a < 3; ++a)
            h[a] += (3.0 * mr * r[a] - mq[a]) * inv3;
    }
    const double vol = cp[0] * atom_volume;
    for (int a = 0; a < 3; ++a)
        out[a] = ORC_MU0_OVER_4PI * h[a] - (4.0 * ORC_PI * ORC_MU0_OVER_4PI / 3.0) * cp[5 + a] / vol;
}

int orc_demag_update(const orc_system *s, const double *S)
{
    orc_demag *d = s->demag;
    const int64_t n = s->n;
    if (!d || n <= 0)
        return 0;
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *acc = NULL;
    int64_t n_mc = 0;
    if (!cell || bin_cells(s, S, cell, &acc, &n_mc) != 0) {
        free(cell);
        return -2;
    }
    double *Hc = (double *)calloc((size_t)n_mc * 3, sizeof(double));
    if (!Hc) {
        free(acc);
        free(cell);
        return -2;
    }
    for (int64_t p = 0; p < n_mc; ++p)
        cell_field(acc, n_mc, p, d->atom_volume, Hc + 3 * p);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            d->field[3 * i + a] = Hc[3 * cell[i] + a];
    d->n_cells = n_mc;
    d->valid = 1;
    free(acc);
    free(Hc);
    free(cell);
    return 0;
}

int orc_demag_sample(const orc_system *s, const double *S, int64_t n_sites, const int64_t *sites, double *out)
{
    const orc_demag *d = s->demag;
    const int64_t n = s->n;
    if (!d || n <= 0)
        return -1;
    for (int64_t k = 0; k < n_sites; ++k)
        if (sites[k] < 0 || sites[k] >= n)
            return -1;
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *acc = NULL;
    int64_t n_mc = 0;
    if (!cell || bin_cells(s, S, cell, &acc, &n_mc) != 0) {
        free(cell);
        return -2;
    }
    for (int64_t k = 0; k < n_sites; ++k)
        cell_field(acc, n_mc, cell[sites[k]], d->atom_volume, out + 3 * k);
    free(acc);
    free(cell);
    return 0;
}

/*
 * sllg_oracle.h -- plain, single-threaded FP64 reference implementation of
 * the stochastic Landau-Lifshitz-Gilbert (sLLG) spin dynamics integrated
 * with the Heun predictor-corrector scheme, and of Metropolis Monte Carlo
 * with Hinzke-Nowak trial moves, as described in Evans et al.,
 * "Atomistic spin model simulations of magnetic nanomaterials"
 * (J. Phys.: Condens. Matter 26, 103202 (2014); arXiv:1310.6143).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library
 * against the paper.  It is slow on purpose: one thread, IEEE double,
 * no FMA contraction, no reordering of the paper's steps.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the product path never does.  It shares no code with the GPU library.
 *
 * Units are SI as in Table 1 of the paper: moments in J/T, exchange in
 * joules per link, anisotropy in joules per atom, fields in tesla, time in
 * seconds, temperature in kelvin.
 */
#ifndef SLLG_ORACLE_H
#define SLLG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boltzmann constant and Bohr magneton, Table 1 of the paper. */
#define ORC_KB 1.3807e-23
#define ORC_MUB 9.2740e-24

/* Macrocell demagnetising field ("Demagnetising fields"; see demag.c).
 * pos: [3n] atom positions in metres; cell_size: macrocell edge (m);
 * atom_volume: unit-cell volume / atoms per unit cell (m^3); every: steps
 * between updates.  field ([3n], caller-owned) holds the field of the last
 * update, per atom (tesla); valid says whether it holds one.  A Heun step
 * numbered k first recomputes it from the current spins when k is a
 * multiple of `every` or no field is held, then uses it, unchanged, in
 * predictor and corrector.  The energy records leave it out. */
typedef struct {
    const double *pos;
    double cell_size;
    double atom_volume;
    int64_t every;
    double *field;
    int valid;
    int64_t n_cells;    /* set by the update */
} orc_demag;

/* A spin system in the form the Hamiltonian section writes it.
 * Every per-site array has n entries (easy_axis has 3n).  The neighbour
 * list is CSR: the entries of row i are row_ptr[i] .. row_ptr[i+1]-1, with
 * neighbour col[k] coupled by J[ntype[k]] (ntype may be NULL: all type 0).
 * With J_tensor (n_types x 9, row-major) the coupling of a link of type t
 * is the matrix J_tensor[t] instead of J[t] (tensorial exchange; the
 * reverse link must carry the transposed matrix).  k_c (n entries, may be
 * NULL) adds cubic anisotropy (k_c/2)(Sx^4 + Sy^4 + Sz^4) per site. */
typedef struct {
    int64_t n;
    const int64_t *row_ptr;
    const int32_t *col;
    const uint8_t *ntype;
    const double *J;
    int n_types;
    const double *mu_s;
    const double *k_u;
    const double *easy_axis;
    double alpha;          /* microscopic (Gilbert) damping lambda */
    double gamma;          /* gyromagnetic ratio, 1/(T s) */
    double dt;             /* time step, s */
    double temperature;    /* K */
    double H[3];           /* applied field, T */
    uint64_t seed;         /* Philox key */
    const double *J_tensor;  /* NULL: scalar exchange J[type] */
    const double *k_c;       /* NULL: no cubic anisotropy */
    orc_demag *demag;        /* NULL: no demagnetising field */
} orc_system;

/* Recompute the demagnetising field from the spins S (0, or -2 when out of
 * memory). */
int orc_demag_update(const orc_system *s, const double *S);
/* The same field at the cells of the given sites only (out: 3 per site), the
 * held field left untouched: for spot checks of large systems.  0, -1 for a
 * site out of range or no demagnetising field, -2 when out of memory. */
int orc_demag_sample(const orc_system *s, const double *S, int64_t n_sites, const int64_t *sites, double *out);

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox_batch(int64_t count, const uint32_t *ctr, const uint32_t *key, uint32_t *out);

/* Three standard normals for (site, step): Philox counter
 * (site, step low word, step high word, purpose), key = seed, then two
 * Box-Muller pairs of which the fourth normal is dropped. */
void orc_gaussian3(uint64_t seed, uint64_t step, uint64_t site, uint32_t purpose, double g[3]);
void orc_gaussian3_batch(uint64_t seed, uint64_t step, int64_t count, const uint64_t *sites,
                         uint32_t purpose, double *g);

/* Fields (tesla) and the right-hand side of the LLG equation. */
void orc_exchange_field(const orc_system *s, const double *S, int64_t i, double h[3]);
void orc_effective_field(const orc_system *s, const double *S, int64_t i, double h[3]);
void orc_effective_fields(const orc_system *s, const double *S, double *H_out);
void orc_llg_rhs(double gamma, double alpha, const double spin[3], const double h[3], double ds[3]);
double orc_thermal_sigma(const orc_system *s, int64_t i);

/* Observables. */
double orc_energy(const orc_system *s, const double *S);
void orc_magnetisation(const orc_system *s, const double *S, double m[3]);

/* One Heun step numbered `step` (used as the noise counter).  S (3n) is
 * updated in place; work must hold 9n doubles.  Returns 0, or -1 if a spin
 * could not be normalised (zero length or not finite). */
int orc_heun_step(const orc_system *s, double *S, uint64_t step, double *work);

/* n_steps Heun steps numbered step0, step0+1, ...  After every step the
 * reduced magnetisation (3 values) and the energy are written to m_out and
 * E_out when those are not NULL.  Returns 0, -1 on a bad spin, -2 on
 * allocation failure. */
int orc_integrate(const orc_system *s, double *S, uint64_t step0, int64_t n_steps,
                  double *m_out, double *E_out);

/* Zero-temperature relaxation: Heun steps until every spin's torque
 * |S x H| is at most torque_tol (tesla), or max_steps.  Returns the number
 * of steps taken, or -1 if max_steps was reached first. */
int64_t orc_relax(const orc_system *s, double *S, double torque_tol, int64_t max_steps,
                  uint64_t step0);
double orc_max_torque(const orc_system *s, const double *S);

/* Monte Carlo ("Monte Carlo Methods", Hinzke-Nowak moves; see mc.c for the
 * colour-class sweep order and the random-number layout).
 * orc_greedy_colours: colour[i] = the smallest colour not taken by a
 * neighbour j < i; returns the number of colours (-1 on allocation failure).
 * orc_greedy_colours_in: the same with the sites visited in the order
 * visit[0..n-1] (a permutation; NULL: ascending), each taking the smallest
 * colour no neighbour visited before it has.
 * orc_lattice_visit: the visiting order of a lattice of nb sites per cell,
 * site i = b + nb (x + cells[0] (y + cells[1] z)): sites grouped by basis
 * site b, then by the parity of x + y + z, ascending within a group (0, or
 * -1 when nb x cells != n).
 * orc_mc_cone_width: sigma_g = (2/25)(kB T/muB)^(1/5).
 * orc_mc_choice: move type (0 flip, 1 Gaussian, 2 random) and acceptance
 * uniform of (site, step).
 * orc_mc_trial: one trial on spin i at Monte Carlo step `step`; returns 1
 * when accepted.  orc_mc_step: one step (every site once, colour by colour);
 * returns the number of accepted trials.  orc_mc_run: n_steps steps
 * numbered step0, step0+1, ...; m, E and the accepted count after each
 * step go to the arrays that are not NULL.  Returns 0 or -2.
 * orc_mc_run_visit: orc_mc_run with the colour classes of
 * orc_greedy_colours_in(visit).
 * orc_mc_step_random / orc_mc_run_random: the same in the paper's order, N
 * trials on sites drawn at random with replacement. */
int orc_greedy_colours(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *colour);
int orc_greedy_colours_in(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *visit,
                          int32_t *colour);
int orc_lattice_visit(int64_t n, int nb, const int cells[3], int64_t *visit);
double orc_mc_cone_width(double temperature);
void orc_mc_choice(uint64_t seed, uint64_t step, uint64_t site, uint32_t *move, double *u);
int orc_mc_trial(const orc_system *s, double *S, int64_t i, uint64_t step);
int64_t orc_mc_step(const orc_system *s, double *S, const int32_t *colour, int n_colours, uint64_t step);
int orc_mc_run(const orc_system *s, double *S, uint64_t step0, int64_t n_steps, double *m_out,
               double *E_out, int64_t *accepted_out);
int orc_mc_run_visit(const orc_system *s, const int64_t *visit, double *S, uint64_t step0, int64_t n_steps,
                     double *m_out, double *E_out, int64_t *accepted_out);
int64_t orc_mc_step_random(const orc_system *s, double *S, uint64_t step);
int orc_mc_run_random(const orc_system *s, double *S, uint64_t step0, int64_t n_steps, double *m_out,
                      double *E_out, int64_t *accepted_out);

/* Brute-force neighbour search over all pairs (minimum image on the axes
 * with box[a] > 0).  A pair at distance r with shell_lo[t] <= r <= shell_hi[t]
 * becomes a link of type t.  Rows come out with ascending columns.
 * Pass row_ptr (n+1) and col/ntype with room for cap entries; returns the
 * number of entries, or -1 if cap is too small. */
int64_t orc_neighbours(int64_t n, const double *pos, const double box[3], int n_shells,
                       const double *shell_lo, const double *shell_hi,
                       int64_t *row_ptr, int32_t *col, uint8_t *ntype, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif

/*
 * sllg.h -- C ABI of libsllg: stochastic Landau-Lifshitz-Gilbert spin
 * dynamics of a classical Heisenberg system, integrated with the Heun
 * predictor-corrector scheme on an AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Evans et al., "Atomistic spin model simulations
 * of magnetic nanomaterials" (J. Phys.: Condens. Matter 26, 103202 (2014),
 * arXiv:1310.6143).  Section names below refer to that paper.
 *
 * Conventions for every call
 *  - Units are SI (Table 1): moments mu_s in J/T, exchange J in joules per
 *    link, anisotropy k_u in joules per atom, fields in tesla, time in
 *    seconds, temperature in kelvin, energies in joules.
 *  - Pointers named *_dev are device (HBM) pointers on the system's GPU; all
 *    other array pointers are host pointers.
 *  - Host inputs are copied during the call; the caller keeps ownership and
 *    may free them on return.  Outputs go to caller-owned buffers.
 *    Handles belong to the library until the matching destroy call.
 *  - Every call returns an sllg_status.  On failure the handle is left as it
 *    was before the call (except where a call says otherwise) and
 *    sllg_last_error() holds a message.  No C++ exception crosses the ABI.
 *  - A handle must not be used from two threads at the same time.
 *  - `stream` is a hipStream_t on the system's device, or NULL for the
 *    library's own stream.  Calls that take a stream return when the work
 *    is finished (host outputs are complete).
 */
#ifndef SLLG_H
#define SLLG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLLG_OK = 0,
    SLLG_E_ARG = -1,        /* an argument is invalid (range, shape, NaN, ...) */
    SLLG_E_NOMEM = -2,      /* device or host allocation failed */
    SLLG_E_DEVICE = -3,     /* a HIP runtime call failed */
    SLLG_E_STATE = -4,      /* call not valid in the current state (e.g. not set up, not ready) */
    SLLG_E_BUDGET = -5,     /* request does not fit the server's HBM budget */
    SLLG_E_NUMERIC = -6,    /* the dynamics produced a non-finite value */
    SLLG_E_CANCELLED = -7   /* the request was cancelled */
} sllg_status;

typedef enum { SLLG_FP32 = 0, SLLG_FP64 = 1 } sllg_precision;

typedef struct sllg_system sllg_system;

/* ---------------------------------------------------------------------------
 * System set-up: the spin Hamiltonian (section "The classical spin
 * Hamiltonian"), H = -sum_{i!=j} J_ij S_i.S_j - sum_i k_u (S_i.e_i)^2
 *                    - sum_i mu_s S_i.H_app.
 * ------------------------------------------------------------------------- */

/* Create an empty system of n_spins spins on HIP device `device`.
 * precision: SLLG_FP32 stores and integrates spins in single precision (the
 * magnetisation and energy reductions are always double); SLLG_FP64 does
 * everything in double.  1 <= n_spins < 2^28.  *out receives the handle.
 * The device is opened at the first call that needs it (integration,
 * measurement, reading spins back after integrating); set-up calls only
 * validate and copy on the host.  Until sllg_set_spins every spin points
 * along +z; the noise seed and step counter start at 0. */
sllg_status sllg_create(int device, sllg_precision precision, int64_t n_spins, sllg_system **out);

/* Release a system and all its device memory.  NULL is ignored. */
void sllg_destroy(sllg_system *sys);

/* Message describing the last failure on this handle ("" if none).  The
 * string stays valid until the next call on the handle.  NULL -> message of
 * the last failed sllg_create in this thread. */
const char *sllg_last_error(const sllg_system *sys);

/* Name of a status code. */
const char *sllg_status_string(sllg_status status);

/* Interaction list (section "Atomistic system generation": the per-atom
 * list of exchange partners) in CSR form.  row_ptr[n+1] (row_ptr[0] = 0,
 * non-decreasing); col[row_ptr[n]] neighbour indices in [0, n), no self
 * links; ntype[row_ptr[n]] interaction types in [0, n_types), or NULL for
 * all type 0; J[n_types] exchange constants in joules per link, 1 <= n_types
 * <= 16.  At most 4095 neighbours per site (long-range exchange: the paper
 * notes hundreds of partners per atom).  Each link must appear in both
 * rows with the same J (the pair sum runs over i != j with J_ij = J_ji);
 * this is checked unless the option "check_symmetry" is 0.  The exchange
 * field on spin i is (1/mu_s,i) sum_k J[ntype[k]] S[col[k]].  A new
 * neighbour list drops exchange tensors set before it. */
sllg_status sllg_set_neighbours(sllg_system *sys, const int64_t *row_ptr, const int32_t *col,
                                const uint8_t *ntype, const double *J, int n_types);

/* Convenience builders of the paper's test structures (appendix
 * "Atomistic system generation": a unit cell replicated on a grid of cells,
 * optionally cut to a shape, every site's exchange partners from the cell's
 * neighbour template) as CSR lists for sllg_set_neighbours.  Host only, no
 * device and no handle; errors go to sllg_last_error(NULL).  Rows are
 * sorted by column, then type.  Two calls: with row_ptr, col, type and pos
 * all NULL they store the number of sites in *n and of links in *nnz; then,
 * with *n and *nnz unchanged, they fill the caller's row_ptr[n + 1],
 * col[nnz] and, when not NULL, type[nnz] and pos[3n] (site positions in
 * units of the cubic cell edge a).  SLLG_E_ARG for NULL n or nnz, bad
 * sizes, counts that differ from the first call's, or more than 2^28 - 1
 * sites; SLLG_E_NOMEM when host memory runs out.
 *
 * sllg_build_sc: simple cubic, cells[0] x cells[1] x cells[2] sites, site
 * i = x + cells[0] (y + cells[1] z), the 6 nearest neighbours (type 0);
 * periodic[a] != 0 wraps axis a (which then needs at least 3 cells).
 * sllg_build_bcc: body-centred cubic, 2 sites per cell, i = b + 2 (x +
 * cells[0] (y + cells[1] z)) with b = 0 at the cell corner and b = 1 at its
 * centre: the 8 first neighbours at a sqrt(3)/2 (type 0) and, with
 * second_neighbours != 0, the 6 second neighbours at a (type 1).  Both
 * number their sites as sllg_set_lattice declares them (n_basis 1 or 2), so
 * the block can take the fused step.
 * sllg_build_fcc_sphere: a sphere cut from an fcc crystal of lattice
 * constant a_nm, centred on a site: the sites (x, y, z) a/2 with x + y + z
 * even at most radius_nm + 1e-9 nm from the centre, numbered by z, then y,
 * then x; the 12 nearest neighbours at a / sqrt(2) inside the sphere
 * (type 0), fewer at the surface. */
sllg_status sllg_build_sc(const int cells[3], const int periodic[3], int64_t *n, int64_t *nnz, int64_t *row_ptr,
                          int32_t *col, uint8_t *type, double *pos);
sllg_status sllg_build_bcc(const int cells[3], const int periodic[3], int second_neighbours, int64_t *n,
                           int64_t *nnz, int64_t *row_ptr, int32_t *col, uint8_t *type, double *pos);
sllg_status sllg_build_fcc_sphere(double a_nm, double radius_nm, int64_t *n, int64_t *nnz, int64_t *row_ptr,
                                  int32_t *col, uint8_t *type, double *pos);

/* Lattice numbering (section "Atomistic system generation": a unit cell of
 * n_basis sites replicated on a grid of cells[0] x cells[1] x cells[2]
 * cells).  Declares that site i of the current neighbour list is basis site
 * b of cell (x, y, z) with i = b + n_basis (x + cells[0] (y + cells[1] z));
 * periodic[a] != 0 marks axis a as periodic.  Every link must join cells at
 * most one cell apart on each axis (across the boundary on a periodic
 * axis); SLLG_E_ARG otherwise, or when n_basis x cells does not equal the
 * number of spins.  The declaration lets the library run the fused step: a
 * single launch per Heun step in which each workgroup recomputes the
 * predictor on a ring of cells around its tile, so that every predictor of
 * its sites' neighbours is ready before its correctors, the order the
 * section "Time Integration of the LLG Equation" requires.  The fused step
 * takes lattices periodic in x and y (z periodic or open) with at most 2
 * sites per cell whose links depend only on the plane and the basis site,
 * uniform materials, scalar exchange, no cubic anisotropy or demagnetising
 * field; in FP64 only lattices whose sites all have the simple-cubic or bcc
 * links (sllg_get_option "lattice" = 2 when the structure qualifies,
 * "fused_active" = 1 when the next integration takes it); other systems run
 * the two-launch step.  The exchange sum of a site is then added in a fixed
 * order (links into the plane below, its own plane, the plane above), so
 * trajectories agree with the two-launch step to rounding, not bit for
 * bit.  Call after sllg_set_neighbours; a new
 * neighbour list drops the declaration.  SLLG_E_STATE before
 * sllg_set_neighbours. */
sllg_status sllg_set_lattice(sllg_system *sys, int n_basis, const int cells[3], const int periodic[3]);

/* Atomic moments mu_s (J/T, > 0), uniaxial anisotropy constants k_u
 * (J/atom, any sign) and easy axes e (unit vectors, normalised here).
 * per_site = 0: one value each (mu_s[1], k_u[1], easy_axis[3]) for every
 * site; per_site = 1: mu_s[n], k_u[n], easy_axis[3n].  At most 256 distinct
 * (mu_s, k_u) pairs, (mu_s, k_u, k_c) triples with sllg_set_cubic_anisotropy
 * (whose constants are kept when the materials are set again).  Section
 * "The classical spin Hamiltonian", uniaxial anisotropy; anisotropy field
 * 2 k_u / mu_s. */
sllg_status sllg_set_materials(sllg_system *sys, const double *mu_s, const double *k_u,
                               const double *easy_axis, int per_site);

/* Tensorial exchange (section "The classical spin Hamiltonian": the exchange
 * interaction as a 3x3 tensor; its antisymmetric off-diagonal part is the
 * Dzyaloshinskii-Moriya interaction).  J[n_types][3][3] row-major, joules
 * per link, for the types of the current neighbour list (n_types must
 * match it); replaces the scalar J of those types.  A link i -> j of type t
 * contributes -S_i^T J[t] S_j to the energy once; the field on spin i is
 * (1/mu_s,i) sum_k J[ntype[k]] S[col[k]] (matrix times vector).  The
 * reverse link j -> i must carry the transpose: checked against the types
 * the symmetry check of sllg_set_neighbours found on reverse links (not
 * checked when "check_symmetry" was 0).  The library copies J.  J = NULL
 * returns to the scalar table.  Errors: SLLG_E_STATE before
 * sllg_set_neighbours; SLLG_E_ARG for a count mismatch, a non-finite
 * entry or a tensor that is not the transpose of its reverse type's.
 * Not available to serving requests. */
sllg_status sllg_set_exchange_tensors(sllg_system *sys, const double *J, int n_types);

/* Cubic anisotropy (section "The classical spin Hamiltonian": energy
 * (k_c/2)(Sx^4 + Sy^4 + Sz^4) per atom along the crystal axes x, y, z;
 * field -(2 k_c/mu_s)(Sx^3, Sy^3, Sz^3)).  k_c in J/atom, any sign:
 * per_site = 0 one value for every site, 1 one per site (k_c[n]); combined
 * with the materials of sllg_set_materials (whichever call comes last), at
 * most 256 distinct (mu_s, k_u, k_c).  k_c = NULL removes it.  Errors:
 * SLLG_E_STATE before sllg_set_materials; SLLG_E_ARG for a non-finite
 * value.  Not available to serving requests. */
sllg_status sllg_set_cubic_anisotropy(sllg_system *sys, const double *k_c, int per_site);

/* Macrocell demagnetising field (section "Demagnetising fields").  pos[3n]:
 * atom positions in metres; the sample is cut into cubic macrocells of edge
 * cell_size (m) on a grid that starts a thousandth of a cell below the
 * smallest coordinate on each axis (atomic planes on a cell boundary belong
 * to the upper cell); only cells holding atoms take part.  Cell moment
 * m_p = sum mu_s,i S_i; cell position = magnetic centre of mass
 * sum mu_s,i x_i / sum mu_s,i; cell volume = atoms * atom_volume (unit-cell
 * volume / atoms per unit cell, m^3).  Field of cell p:
 * mu0/(4 pi) sum_{q != p} [3 (m_q . r) r - m_q] / |x_q - x_p|^3
 * - (mu0/3) m_p / V_p (r the unit vector from p to q), added to the
 * effective field of every atom of the cell.  It is recomputed from the
 * current spins before every step whose number is a multiple of `every`
 * (and before the first step after it was set, after sllg_set_spins or
 * sllg_restore, or after an option that rebuilds the device state), then
 * held, the same in predictor and corrector.  The energy records leave it
 * out.  Monte Carlo refuses a system with it (SLLG_E_STATE).  pos = NULL
 * switches it off; a new neighbour list drops it.  The library copies pos.
 * Errors: SLLG_E_STATE before sllg_set_neighbours; SLLG_E_ARG for
 * non-finite positions, cell_size or atom_volume <= 0, every < 1.  Not
 * available to serving requests. */
sllg_status sllg_set_demag(sllg_system *sys, const double *pos, double cell_size, double atom_volume,
                           int64_t every);

/* Write the demagnetising field in effect per atom into field_out[3n]
 * (tesla): the field held since the last scheduled update (every `every`
 * steps, Section "Demagnetising field"), so that reading it never changes
 * the trajectory; when no field is held yet (after sllg_set_demag or
 * sllg_set_spins) the field of the current spins, computed now and held as
 * a scheduled update would hold it.  SLLG_E_STATE without sllg_set_demag. */
sllg_status sllg_demag_field(sllg_system *sys, double *field_out, void *stream);

/* Damping lambda >= 0, gyromagnetic ratio gamma > 0 (1/(T s); Table 1 gives
 * 1.76e11) and time step dt > 0 (s).  Section "Spin Dynamics" (atomistic LLG
 * equation) and "Time Integration of the LLG Equation". */
sllg_status sllg_set_integrator(sllg_system *sys, double alpha, double gamma, double dt);

/* Temperature T >= 0 (K) of the Langevin heat bath (section "Langevin
 * Dynamics": thermal field of width sqrt(2 lambda kB T / (gamma mu_s dt)))
 * and applied field H_app[3] (T). */
sllg_status sllg_set_conditions(sllg_system *sys, double temperature, const double H_app[3]);

/* Noise stream: the thermal field of site i at step n is drawn from
 * Philox4x32-10 with counter (i, n mod 2^32, n div 2^32, 0) and key
 * (seed mod 2^32, seed div 2^32), turned into three normals by Box-Muller.
 * `step` is the number of the next step; every integrated step increments
 * it, so chunked integration equals one long call. */
sllg_status sllg_set_rng(sllg_system *sys, uint64_t seed, uint64_t step);
sllg_status sllg_get_step(const sllg_system *sys, uint64_t *step);

/* Spin directions S[3n] (x, y, z per site).  Each must have finite, non-zero
 * length; they are normalised here. */
sllg_status sllg_set_spins(sllg_system *sys, const double *S);
sllg_status sllg_get_spins(sllg_system *sys, double *S_out);

/* ---------------------------------------------------------------------------
 * Integration: Heun scheme (section "Time Integration of the LLG Equation").
 * Each step: predictor S' = S + dS dt on every spin and renormalisation;
 * effective field re-evaluated at S' with the same thermal field; corrector
 * S <- S + (dS + dS')/2 dt and renormalisation.
 * ------------------------------------------------------------------------- */

/* Advance n_steps >= 0 steps.  After every step the reduced magnetisation
 * m = sum mu_s S / sum mu_s is written to m_out[3*t..3*t+2] and the energy
 * of the Hamiltonian above (thermal field excluded, each link once) to
 * E_out[t], if those pointers are not NULL.  Returns SLLG_E_NUMERIC if an
 * energy came out non-finite or a step produced a non-finite spin (every
 * new spin is checked by the kernel that writes it, records or not; the
 * state is then kept as it is). */
sllg_status sllg_integrate(sllg_system *sys, int64_t n_steps, double *m_out, double *E_out,
                           void *stream);

/* Same, with device output arrays m_dev[3*n_steps] and E_dev[n_steps] (either
 * may be NULL); nothing is copied to the host.  Returns when the work has
 * been queued on `stream`; the outputs are valid once the stream reaches
 * that point.  A non-finite spin (checked on every new spin) sets a flag of
 * the system that is not waited for here: the next sllg_integrate_dev call
 * returns SLLG_E_NUMERIC once the earlier call's work has finished,
 * sllg_integrate and sllg_mc report it at their end, and sllg_get_option
 * "numeric_fault" reads it (waiting for the queued work).  sllg_set_spins
 * and sllg_restore clear it. */
sllg_status sllg_integrate_dev(sllg_system *sys, int64_t n_steps, double *m_dev, double *E_dev,
                               void *stream);

/* Monte Carlo (section "Monte Carlo Methods"): n_steps >= 0 Metropolis
 * steps at the current temperature, field and materials.  A step makes one
 * trial on every site, colour class by colour class of a greedy colouring
 * of the neighbour graph (the sites are visited in ascending order, each
 * taking the smallest colour no earlier-visited neighbour has; with the
 * option "mc_colouring" = 1 on a declared lattice they are visited grouped
 * by basis site and by the parity of the cell's x + y + z, which gives the
 * bcc lattice with first and second neighbours four equal classes; sites
 * of one class share no link, so their trials are made at once).  A trial picks, with probability 1/3 each, a spin flip S' = -S, a
 * Gaussian move S' = |S + sigma_g Gamma| with sigma_g = (2/25)(kB T/muB)^(1/5),
 * or a uniform point on the sphere S' = Gamma/|Gamma| (Hinzke and Nowak),
 * and accepts it if dE <= 0, else if u < exp(-dE/(kB T)).  Random numbers
 * of site i at step k: Gamma from Philox counter (i, k lo, k hi, 2) with
 * Box-Muller as for the thermal field; the move (floor(3 r0 / 2^32)) and u
 * (r1 / 2^32) from counter (i, k lo, k hi, 3).  Steps are numbered by, and
 * advance, the same step counter as the LLG steps.  After every step m and
 * E go to m_out / E_out and the number of accepted trials to
 * accepted_out[t], for the pointers that are not NULL.  The FP64 path
 * takes every decision in double precision, the FP32 path in single. */
sllg_status sllg_mc(sllg_system *sys, int64_t n_steps, double *m_out, double *E_out,
                    int64_t *accepted_out, void *stream);

/* Monte Carlo thermal average (the M(T) protocol of section "Monte Carlo
 * Methods" and "Curie temperature": equilibrate, then average with m and E
 * taken after every step): n_eq steps of sllg_mc, then n_avg steps, and
 * out[9] = { <|m|>, se(<|m|>), <m_x>, <m_y>, <m_z>, <E>, se(<E>),
 * n_blocks, acceptance }.  The averages and standard errors are those of
 * sllg_average over the first n_avg - n_avg % n_blocks steps, in n_blocks
 * (>= 2, <= min(n_avg, 4096)) equal consecutive blocks; acceptance is the
 * accepted trials of all n_avg steps over n * n_avg.  SLLG_E_STATE with a
 * demagnetising field on. */
sllg_status sllg_mc_average(sllg_system *sys, int64_t n_eq, int64_t n_avg, int n_blocks, double out[9],
                            void *stream);

/* Observables of the current state: m[3] and E (either may be NULL). */
sllg_status sllg_measure(sllg_system *sys, double m[3], double *E, void *stream);

/* Thermal average (the M(T) protocol of the paper: equilibrate, then
 * average with the magnetisation sampled every step).  Runs n_eq steps, then
 * n_avg steps, and fills out[8] = { <|m|>, se(<|m|>), <m_x>, <m_y>, <m_z>,
 * <E>, se(<E>), n_blocks }, where se is the standard error of the mean from
 * n_blocks (>= 2, <= n_avg) equal consecutive blocks. */
sllg_status sllg_average(sllg_system *sys, int64_t n_eq, int64_t n_avg, int n_blocks,
                         double out[8], void *stream);

/* Temperature ramp with continuation (section "Curie temperature": each
 * point starts from the final state of the previous one): for each of the
 * n_points temperatures T[k], set T, then sllg_average(n_eq, n_avg).
 * out[8*k .. 8*k+7] receives the point's averages. */
sllg_status sllg_sweep_temperature(sllg_system *sys, const double *T, int64_t n_points,
                                   int64_t n_eq, int64_t n_avg, int n_blocks, double *out,
                                   void *stream);

/* Field sweep with continuation (hysteresis loop): for each applied field
 * H[3*k .. 3*k+2], set it and run sllg_average(n_eq, n_avg); out as above. */
sllg_status sllg_sweep_field(sllg_system *sys, const double *H, int64_t n_points, int64_t n_eq,
                             int64_t n_avg, int n_blocks, double *out, void *stream);

/* Largest torque max_i |S_i x H_i| (tesla) of the current state, with the
 * deterministic effective field (exchange, anisotropy, applied field; no
 * thermal term).  Section "Angular variation of the Coercivity": the
 * convergence measure of the quasi-static solution. */
sllg_status sllg_max_torque(sllg_system *sys, double *torque_out, void *stream);

/* Quasi-static relaxation (section "Angular variation of the Coercivity":
 * the LLG equation is solved at zero temperature until the torque on the
 * system is at most 1e-6 T, a local energy minimum).  Heun steps with the
 * system's damping and dt, continuing the step counter; the largest torque
 * is checked before the first step and then after every check_every steps
 * (check_every = 1 stops at the first step that reaches torque_tol).
 * steps_out: steps taken, or -1 when max_steps were taken without reaching
 * the tolerance (status SLLG_E_NUMERIC then); torque_out: the last value
 * checked.  Either may be NULL.  Errors: SLLG_E_STATE when the temperature
 * is not 0; SLLG_E_ARG for tol < 0, max_steps < 0 or check_every < 1. */
sllg_status sllg_relax(sllg_system *sys, double torque_tol, int64_t max_steps, int64_t check_every,
                       int64_t *steps_out, double *torque_out, void *stream);

/* Quasi-static hysteresis loop (the same test: the field is changed in
 * steps and the spins relaxed again after each): for each applied field
 * H[3*k .. 3*k+2], set it, sllg_relax, then the reduced magnetisation of the
 * relaxed state into m_out[3*k .. 3*k+2] and the steps taken into
 * steps_out[k] (-1 where max_steps did not suffice; may be NULL).  Several
 * uncoupled spins with per-site easy axes give loops at several angles
 * between field and easy axis in one run. */
sllg_status sllg_hysteresis(sllg_system *sys, const double *H, int64_t n_points, double torque_tol,
                            int64_t max_steps, int64_t check_every, double *m_out, int64_t *steps_out,
                            void *stream);

/* Launch-shape autotuner: times every candidate launch configuration, the
 * best of two runs of trial_steps (2..100000) steps of this system each,
 * keeps the fastest and writes its time per step (us) to *us_per_step (may
 * be NULL).  With the fused step active ("fused_active" 1) the candidates
 * are the eight fused shapes (tile, planes per item, threads per
 * workgroup) the occupancy and traffic model ranks best; otherwise every
 * tile size of the two-launch step ("tile_sites": 512, 1024, 2048 in FP32;
 * 512, 1024 in FP64), each with its launch shapes ("lds_window" 1 or 0;
 * "tile_order" 1 or 0; XCD mappings 0, 1, 2 of "xcd_remap"; 1/2, 1 or 2
 * resident grids of workgroups per launch).  Systems under 2^20 spins also
 * try 16, 64 or 256 steps per captured HIP graph.  The spins, the step
 * counter, the held demagnetising field and every result stay exactly as
 * they were.  Launch shapes do not change the arithmetic of a spin; the m
 * and E records (FP64 sums of per-tile or per-workgroup partial sums) may
 * change at FP64 rounding when the tile size or shape changes.  The choice
 * can be read back with sllg_get_option ("fused_tile_x", "fused_tile_y",
 * "fused_planes", "fused_threads"; "tile_sites", "lds_window",
 * "tile_order", "xcd_remap", "grid_scale_pct"; "graph_steps",
 * "tuned_ns_per_step").  Setting
 * SLLG_AUTOTUNE_LOG=1 in the environment prints every candidate's time to
 * stderr. */
sllg_status sllg_autotune(sllg_system *sys, int trial_steps, double *us_per_step, void *stream);

/* Thermal normals Gamma[3n] of sites 0..n-1 at step `step`, drawn exactly as
 * the step kernels of the given precision draw them (Philox counter and
 * Box-Muller as in sllg_set_rng), copied to the host array out.  For
 * checking the noise stream; 1 <= n < 2^28. */
sllg_status sllg_thermal_normals(int device, sllg_precision precision, uint64_t seed, uint64_t step,
                                 int64_t n, double *out);

/* sllg_thermal_normals without device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same normals, bit for bit, staged in a fixed
 * scratch of 2^18 sites (6 MiB) that the library holds on every device it
 * has run this call on until the process ends, instead of a buffer
 * allocated per call.  1 <= n <= 2^18 (SLLG_E_ARG beyond, with the reason
 * in sllg_last_error(NULL)).  Runs on the device's null stream and copies
 * to the host array out[3n] before returning.  Calls that overlap on one
 * device share its scratch and race; calls on different devices do not.
 * Nothing in the scratch needs clearing: each call writes every value it
 * reads back. */
sllg_status sllg_thermal_normals_noalloc(int device, sllg_precision precision, uint64_t seed, uint64_t step,
                                         int64_t n, double *out);

/* ---------------------------------------------------------------------------
 * Checkpoint / resume.  The state is the spins, the noise seed, the step
 * counter and, with a demagnetising field on, the field held since its last
 * scheduled update; because the noise is counter-based, a restored run
 * continues exactly as the uninterrupted one would.  Restoring needs a
 * system set up the same way (sites, precision, demagnetising field on or
 * off); a blob written without a held field leaves the field to be
 * computed at the next step.
 * ------------------------------------------------------------------------- */
sllg_status sllg_checkpoint_size(const sllg_system *sys, size_t *bytes);
sllg_status sllg_checkpoint(sllg_system *sys, void *buf, size_t bytes);
sllg_status sllg_restore(sllg_system *sys, const void *buf, size_t bytes);

/* Tuning and behaviour options (integers):
 *   "check_symmetry"  1 (default) / 0: verify J_ij = J_ji in set_neighbours
 *   "graph_steps"     steps per captured HIP graph chunk, 0 = no graphs
 *                     (default: chosen from the system size)
 *   "xcd_remap"       tile order of the step launches: 1 (default) each XCD
 *                     sweeps one contiguous range of tiles,
 *                     interleaved over its workgroups; 2 the same ranges cut
 *                     into one contiguous run per workgroup; 0 plain
 *                     grid-stride order
 *   "grid_scale_pct"  workgroups per step launch, in % of the resident grid
 *                     (10..800, default 100)
 *   "tile_order"      1 (default): when the stencil's far links point about
 *                     one lattice plane away, list the tiles as groups of
 *                     "tile_group" adjacent columns swept plane by plane (a
 *                     tile's far neighbours were read a few tiles earlier
 *                     and are still cached); 0 site order
 *   "tile_group"      tile columns per group for tile_order 1 (1..4096;
 *                     0, the default, sizes the groups from the L2 capacity)
 *   "lds_window"      1 (default): a workgroup copies its tile's spins and a
 *                     halo into LDS and reads near neighbours from there; 0:
 *                     every neighbour and the site's own spin are read from
 *                     global memory (can be faster for small, cache-resident
 *                     systems).  Results are the same bit for bit.
 *   "tile_sites"      consecutive sites one workgroup integrates together:
 *                     0 (default) = from the system size (the largest tile,
 *                     2048 in FP32 / 1024 in FP64, halved down to 512 until
 *                     the system has at least 2048 tiles), or a power of two
 *                     in that range.  Trajectories do not depend on it; the
 *                     m and E records do at the level of FP64 rounding (the
 *                     tile is the first level of their summation tree).  The
 *                     server always uses the largest tile.
 *   "stencil"         1 (default) / 0: let the next sllg_set_neighbours store
 *                     the list as per-site stencil patterns when at most 256
 *                     distinct (column - row, type) rows occur (<= 1024
 *                     entries in all, tables in LDS), else as wide stencil
 *                     patterns when at most 65535 occur (<= 2^22 entries
 *                     with every pattern padded to the longest; tables in
 *                     global memory: periodic long-range lattices); 0 keeps
 *                     the general SELL-64 form.  The sums are the same in
 *                     every form (near links, then far ones, each in row
 *                     order)
 *   "mc_colouring"    0 (default): the Monte Carlo colouring visits the
 *                     sites in ascending order; 1: on a declared lattice
 *                     (sllg_set_lattice) grouped by basis site b, then by
 *                     the parity of x + y + z of its cell, ascending within
 *                     a group (without a declaration, ascending).  Sets the
 *                     colour classes at once (the chain of sllg_mc depends
 *                     on them; the spins are kept)
 *   "fused"           1 (default): integrate with the fused step when the
 *                     system qualifies (sllg_set_lattice) and has at least
 *                     2^20 spins (smaller systems run faster with the
 *                     two-launch step's shallow launches); 2: whenever it
 *                     qualifies; 0: always the two-launch step
 *   "fused_tile_x", "fused_tile_y", "fused_planes", "fused_threads"
 *                     shape of the fused step's work items: a tile of
 *                     tile_x x tile_y cell columns marched through `planes`
 *                     planes by a workgroup of `threads` (256, 512, or 1024
 *                     for the simple-cubic and bcc kinds in FP32) threads,
 *                     which needs (tile_x + 2)(tile_y + 2) <= threads,
 *                     tile_x, tile_y >= 6, in FP64 tile_x + 4 <= 16 (256
 *                     threads) or 32 (512), and the planes' LDS within the
 *                     device's limit per workgroup; takes effect once all
 *                     four are set (0 returns to the library's choice; the
 *                     autotuner also picks among shapes).  Results do not
 *                     depend on the shape except the m and E records, at FP64
 *                     rounding.
 * sllg_get_option also reads "neighbour_format": 1 stencil, 2 wide stencil,
 * 0 SELL, -1 unset; "mc_colours": the number of Monte Carlo colour classes
 * (-1 unset); "numeric_fault": 1 once a step or Monte Carlo trial
 * produced a non-finite spin since the spins were last set (waits for the
 * queued work);
 * "lattice": 0 none declared, 1 declared, 2 declared and the fused step can
 * take its structure; "fused_active": 1 when the next integration runs the
 * fused step; the fused_* shape keys read the shape in use;
 * "halo": neighbours with |column - row| up to this many
 * sites are read from the tile's window in LDS, the rest from HBM (-1 unset).
 */
sllg_status sllg_set_option(sllg_system *sys, const char *key, int64_t value);
sllg_status sllg_get_option(const sllg_system *sys, const char *key, int64_t *value);

/* ---------------------------------------------------------------------------
 * Serving: many independent systems ("statistical parallelism" of the
 * paper's parallelisation appendix: independent runs for parameter sweeps or
 * seeds) admitted by HBM budget and advanced together by one batched set of
 * kernels, in chunks of steps.  Requests that arrive while others run join
 * at the next chunk boundary (continuous batching).
 * ------------------------------------------------------------------------- */
typedef struct sllg_server sllg_server;

typedef struct {
    size_t hbm_budget;      /* bytes of device memory the server may use for requests */
    int max_active;         /* most requests on the device at once (<= 4096) */
    int chunk_steps;        /* steps per batched launch sequence (even, 2..4096) */
    sllg_precision precision;
} sllg_server_opts;

typedef struct {
    int64_t n_spins;
    const int64_t *row_ptr;   /* CSR as in sllg_set_neighbours */
    const int32_t *col;
    const uint8_t *ntype;     /* or NULL */
    const double *J;
    int n_types;
    const double *mu_s;       /* as in sllg_set_materials */
    const double *k_u;
    const double *easy_axis;
    int per_site;
    const double *S0;         /* initial spins [3n], or NULL for all along +z */
    double alpha, gamma, dt;
    double temperature;
    double H_app[3];
    uint64_t seed;
    int64_t n_steps;          /* >= 1 */
    int64_t n_avg;            /* the last n_avg steps are averaged (0 = none) */
    int record;               /* 1: keep m and E of every step for sllg_fetch */
} sllg_request;

typedef enum {
    SLLG_REQ_QUEUED = 0, SLLG_REQ_RUNNING = 1, SLLG_REQ_DONE = 2,
    SLLG_REQ_FAILED = 3, SLLG_REQ_CANCELLED = 4
} sllg_request_state;

typedef struct {
    int state;                /* sllg_request_state */
    int status;               /* sllg_status of a failed request */
    int64_t n_spins, n_steps, steps_done;
    double m[3], E;           /* final reduced magnetisation and energy */
    double avg[8];            /* averages over the last n_avg steps, as sllg_average */
    double t_submit, t_start, t_done;   /* seconds on the server's clock */
    size_t hbm_bytes;         /* device memory the request holds while it runs */
} sllg_result;

typedef struct {
    int64_t submitted, completed, failed, cancelled, active, queued;
    size_t hbm_in_use, hbm_budget;
    double spin_steps;        /* total spin-steps integrated so far */
    double busy_seconds;      /* time with at least one active request */
    int64_t chunks;           /* batched chunk launches so far */
    /* Launch-shape tuning: each new batch composition (requests that run and
     * their total spins, each bucketed to the next power of two) times the
     * XCD mappings 1, 0, 2 x tile orders 1, 0 on its chunks (results do not
     * depend on them) and keeps the fastest. */
    int64_t tuned_compositions;   /* compositions tuned so far */
    int64_t last_xcd_remap;       /* launch shape of the last chunk */
    int64_t last_tile_order;
} sllg_server_stats;

/* Start a server on `device`.  The server thread owns its own stream. */
sllg_status sllg_server_create(int device, const sllg_server_opts *opts, sllg_server **out);
/* Stop the server thread, cancel outstanding requests, free everything. */
void sllg_server_destroy(sllg_server *srv);
const char *sllg_server_last_error(const sllg_server *srv);
/* Copy a request (inputs are copied) into the queue.  SLLG_E_BUDGET if it
 * could never fit the budget on its own; SLLG_E_ARG if it is malformed. */
sllg_status sllg_submit(sllg_server *srv, const sllg_request *req, uint64_t *ticket);
/* Result so far; SLLG_OK always for a known ticket (check result->state). */
sllg_status sllg_poll(sllg_server *srv, uint64_t ticket, sllg_result *result);
/* Block until the request leaves the queue/running states or timeout_s passes
 * (SLLG_E_STATE on timeout). */
sllg_status sllg_wait(sllg_server *srv, uint64_t ticket, double timeout_s, sllg_result *result);
/* Final spins S_out[3n] and, if recorded, m_series[3*n_steps], E_series[n_steps]
 * of a finished request (any pointer may be NULL).  SLLG_E_STATE if not done. */
sllg_status sllg_fetch(sllg_server *srv, uint64_t ticket, double *S_out, double *m_series,
                       double *E_series);
/* Cancel a queued or running request (it stops at the next chunk boundary). */
sllg_status sllg_cancel(sllg_server *srv, uint64_t ticket);
/* Forget a finished request and free its host copies. */
sllg_status sllg_release(sllg_server *srv, uint64_t ticket);
sllg_status sllg_server_get_stats(sllg_server *srv, sllg_server_stats *stats);
/* The server's clock (seconds), the one t_submit/t_start/t_done use. */
double sllg_server_clock(const sllg_server *srv);

#ifdef __cplusplus
}
#endif
#endif

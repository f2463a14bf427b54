/*
 * qed_oracle.h -- plain, slow, FP64 CPU oracle of the strong-field QED step of
 * Gonoskov et al., "Extended PIC schemes for physics in ultra-strong laser fields:
 * review and developments" (arXiv:1412.6426).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no code, header, table or constant
 * with the HIP library under paper_1412_6426_amd/; the two are written
 * independently from the paper and compared output by output.
 *
 * Units (normalised with a reference angular frequency w_r):
 *   time 1/w_r, length c/w_r, momentum m c, energy m c^2, fields m c w_r / e.
 *   eps_r = hbar w_r / (m c^2); the Sauter-Schwinger field is E_S = 1/eps_r and the
 *   Compton time lambda_C / c = 2 pi eps_r in these units.
 * Species: 0 electron (charge -1), 1 positron (+1), 2 photon (p holds hbar k / (m c)).
 *
 * Parity status of every function is stated in qed_oracle.c next to it.
 */
#ifndef QED_ORACLE_H
#define QED_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_TABLE_N 4096
#define OR_U_LO (-20.0) /* log2 of the smallest tabulated z */
#define OR_U_HI (7.0)   /* log2 of the largest tabulated z; F = 0 beyond */
#define OR_ID_DEAD 0xFFFFFFFFFFFFFFFFull
#define OR_NO_PARENT 0xFFFFFFFFFFFFFFFFull
#define OR_NSUB_MAX 16383
#define OR_NSUB_HIST 32
#define OR_SPECTRUM_BINS 130 /* 10 bins per decade of eps / (m c^2) from 1e-8 */

enum { OR_EXACT = 0, OR_TABLE = 1 };
enum {
  OR_FIELD_UNIFORM = 0,
  OR_FIELD_ROTATING_E = 1,
  OR_FIELD_CP_STANDING = 2,
  OR_FIELD_YEE = 3,
  OR_FIELD_LP_STANDING = 4
};

typedef struct {
  int n;
  double u_lo, u_hi, du;
  double *gA, *gB, *gC; /* e^z * F(z) at z = 2^(u_lo + i du) */
  double s_b0, s_b1, s_c0, s_c1, s_c2; /* small-z series constants */
} or_tables;

typedef struct {
  double *x, *y, *z, *px, *py, *pz, *w;
  uint64_t *id, *parent;
  uint32_t *birth, *n_events; /* n_events may be NULL for photons */
  int64_t count, capacity;
} or_store;

typedef struct {
  int kind;
  double e0[3], b0[3];       /* uniform field */
  double amp, omega, phase;  /* rotating E / CP standing wave amplitude, frequency, phase */
  const float *grid[6];      /* Yee: Ex, Ey, Ez, Bx, By, Bz, each n[2]*n[1]*n[0], x fastest */
  int n[3];
  double dx[3], origin[3];
} or_field;

typedef struct {
  double dt, eps_r, kappa, t0;
  int adaptive, forced_substeps;
  int emission, pairs, push_photons;
  int backend;
  uint64_t seed;
  int64_t step;
  /* Tunable generator factors f_g of Sec. VI for photon emission and pair creation (a value
   * of at most 1 means off).  The event still acts on its parent every time it fires (the
   * lepton recoils, the photon decays); the children of that event are created only with
   * probability 1/f_g, decided by the Philox draw keyed by the parent's id with counter
   * (step, substep | purpose << 16, seed lo, seed hi), purpose 5 (photon) or 6 (pair), first
   * two words as the uniform u, created iff u < 1/f_g, and then carry f_g times the
   * parent's weight. */
  double f_photon, f_pair;
  /* Children in their birth step (Sec. IV.H: several events per iteration).  0: children
   * join the store and are first advanced at the next step.  G > 0: a child born at
   * sub-step k of a parent advanced through T with n_sub sub-steps is advanced in the same
   * step through the rest of it, tau = (n_sub - k - 1) (T / n_sub), with the parent's frozen
   * E, B, its own n_sub over tau, and its own events; children of children likewise, up to G
   * generations.  Children of generation G + 1 wait for the next step. */
  int same_step_generations;
  /* The deterministic form of f_g (Sec. VI, the generator run once every f_g occasions).
   * With f_every set, a factor f_g > 1 must be an integer F, and the children of a parent's
   * event number e (its event count before the event: the n_events column of a lepton, 0
   * for a photon, which has one event) are created iff (e + phi) mod F == 0.  The phase phi
   * in [0, F) is fixed for the parent's life: phi = (o0 F) >> 32 for the first word o0 of
   * the Philox draw keyed by its id with counter (0, 12 << 16, seed lo, seed hi).  Over the
   * phase every event is sampled with probability 1/F, as in the random form, and a parent
   * with n events makes floor(n/F) or ceil(n/F) children. */
  int f_every;
  /* The reverse mode of Sec. VI: the generator runs N_g times at every occasion (a value
   * of at most 1 means off, at most 64; not together with a factor f_g > 1 for the same
   * generator).  Run r draws from counter (step, substep | r << 24, seed lo, seed hi) (run
   * 0 is the ordinary draw) and its children get ids with purpose p | r << 8.  Emission: every
   * run that fires makes a photon of weight w / N_g, with the momentum the lepton had before
   * the sub-step's events; the lepton recoils by the sum of those photon momenta divided by
   * N_g, so that the weighted momentum is conserved event by event.  Pairs: the photon
   * stands for N_g copies of weight w / N_g; every run that fires makes a pair of that
   * weight, the photon keeps (w / N_g) (N_g - m) after m firings in a sub-step and goes on,
   * and is removed when all N_g fire. */
  int runs_photon, runs_pair;
} or_params;

typedef struct {
  int64_t n_start[3];  /* slots of each store at the step start (removed photons included) */
  int64_t advanced[3]; /* particles advanced from the step start: every lepton, and the photons
                          that are alive and have k != 0 */
  int64_t emitted, pairs, dropped, saturated, near_threshold, nsub_near_int, nsub_clamped,
      nonfinite, substeps;
  int64_t nsub_refined;      /* lepton sub-steps taken again at half the length (Sec. IV.H:
                                their length broke Eq. (29) in the state they ended in) */
  int64_t children_advanced; /* children advanced in their birth step (tau > 0) */
  int64_t deferred;          /* children of generation G + 1 created with tau > 0 (dropped ones
                                included), left for the next step */
  double photon_energy;      /* sum of w eps over the emissions (every event, Sec. VI) */
  double max_p_emit;         /* largest emission probability evaluated */
  double max_p_pair;         /* largest pair probability among the decisions that made a pair
                                (every probability >= 1 makes one, so this holds the largest
                                such) */
  int64_t nsub_hist[OR_NSUB_HIST];       /* leptons alive at the step start by n_sub */
  int64_t photon_hist[OR_SPECTRUM_BINS]; /* emissions by photon energy: bin b holds
                                            floor(10 (log10(eps) + 8)) = b, eps in m c^2 */
} or_stats;

/* counter-based generator (Salmon et al., SC'11) */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_uniform(uint32_t lo, uint32_t hi);

/* Bessel-function integrals (DLMF 10.32.9): scaled by e^z */
double or_kint_scaled(double nu, int over_cosh, double z);
double or_A(double z); /* int_z^inf K_{5/3} */
double or_B(double z); /* K_{2/3}(z)        */
double or_C(double z); /* int_z^inf K_{1/3} */
double or_F1(double x);
double or_F2(double x);

int or_tables_build(or_tables *t);
void or_tables_free(or_tables *t);
void or_eval_abc(const or_tables *t, int backend, double z, double *A, double *B, double *C);

double or_rate_emission(const or_tables *t, int backend, double delta, double chi, double gamma,
                        double dtfac);
double or_rate_modified(const or_tables *t, int backend, double r1, double chi, double gamma,
                        double dtfac);
double or_rate_pair(const or_tables *t, int backend, double delta_e, double chi_g, double kabs,
                    double dtfac);

double or_chi_lepton(const double p[3], const double E[3], const double B[3], double eps_r);
double or_chi_photon(const double k[3], const double E[3], const double B[3], double eps_r);
void or_boris(double p[3], double q, double h, const double E[3], const double B[3]);
void or_field_at(const or_field *f, const double x[3], double t, double E[3], double B[3]);
int or_substeps(double dt, double dtq, int *near_int, int *clamped);
double or_dtq_lepton(double chi, double gamma, double eps_r, double kappa);
double or_dtq_photon(double chi_g, double kabs, double eps_r, double kappa);
uint64_t or_child_id(uint64_t parent, uint64_t seed, int64_t step, int substep, int purpose);

int or_step(const or_tables *t, or_store *st /* [3] */, const or_field *f, const or_params *p,
            or_stats *s);

/* Thinning by global even redistribution (Sec. VI): when a store's count (live particles
 * and removed-photon slots) exceeds `trigger` and `target` is below the number of live
 * particles, each live particle is kept with probability q = target / live, decided by
 * the Philox draw keyed by its id with counter (step, 4 << 16, seed lo, seed hi) (first two
 * words as the uniform u; kept iff u < q), and the survivors' weights are multiplied by
 * sum(w of live) / sum(w of kept), so the total weight is unchanged.  Survivors keep their
 * order; removed photons (dead ids) go too.  A store at or below the trigger is not
 * examined (record all zero, factor 1); one examined but not thinned reports its live count
 * and weight.  Parity unpinned for the store order (the GPU fills holes from the tail);
 * the set of survivors and their weights are compared. */
typedef struct {
  int64_t live_before, kept;
  double weight_before, weight_after, factor;
} or_thin_record;
int or_thin(or_store *s, int64_t trigger, int64_t target, uint64_t seed, int64_t step,
            or_thin_record *rec);

/* Thinning per cell (Sec. VI's redistribution applied within a cell; Sec. VII's thinning
 * that caps the particles a cell may hold).  The live particles of the store are grouped
 * by the block of cells that holds them: cell (i, j, k) = floor((x - origin) / dx) per axis,
 * periodic (wrapped into [0, n)); block = cell >> s per axis, s the smallest shift that
 * leaves at most 2^24 - 2 blocks on the n[0] x n[1] x n[2] grid; blocks numbered x fastest;
 * particles with a non-finite coordinate form one more group after every block.  Groups
 * are taken in block order, and the particles of a group in store order.  A group of at
 * most `max_per_cell` particles is kept as it is.  In a larger group of n particles each
 * survives with probability q = max_per_cell / n, decided by the Philox draw keyed by its
 * id with counter (step, 11 << 16, seed lo, seed hi) (first two words as the uniform u;
 * kept iff u < q); if none survives, the one with the smallest u does; the survivors'
 * weights are multiplied by W / K, the group's weight over its survivors' weight (sums in
 * group order), so each group keeps its weight.  The store is rewritten with the survivors
 * in group order (removed photons, is_photon with dead ids, go) and its count set to their
 * number.  rec: live particles before and after, groups (non-empty, removed photons not
 * counted), groups thinned, and the live weight before and after (each the sum over groups
 * in order of the group's sum in order). */
typedef struct {
  int64_t live_before, kept, groups, groups_thinned;
  double weight_before, weight_after;
} or_thin_cells_record;
int or_thin_cells(or_store *s, int is_photon, const int n[3], const double dx[3],
                  const double origin[3], int64_t max_per_cell, uint64_t seed, int64_t step,
                  or_thin_cells_record *rec);

/* The cap on the children one particle generates in one iteration (Sec. VII).  The
 * children born in the last step are the live particles whose birth code (step + 1) << 14 |
 * sub-step names it: birth >> 14 == step, `step` being the step counter after that step,
 * and that have a parent (Schwinger pairs, whose parent is OR_NO_PARENT, are no particle's
 * children).  They are grouped by their parent id.  A group of at most `max_per_parent` children is
 * kept as it is.  In a larger group of n children each survives with probability
 * q = max_per_parent / n, decided by the Philox draw keyed by its id with counter
 * (step, 13 << 16, seed lo, seed hi) (first two words as the uniform u; kept iff u < q); if
 * none survives, those with the smallest u do; the survivors' weights are multiplied by
 * n / K, the group's count over its survivors'.  The children of one parent in one step
 * share its weight (times the generator's factor), so that is the group's weight over its
 * survivors' and each group keeps its weight; only the pairs of one photon in the reverse
 * mode of Sec. VI differ in weight, and keep it in expectation.  Every other particle, and
 * the survivors, keep their store order; the count becomes the number left.  rec: the
 * children, their parents (groups), the groups thinned, the children kept, and the
 * children's weight before and after (sums in store order). */
typedef struct {
  int64_t children, groups, groups_thinned, kept;
  double weight_before, weight_after;
} or_thin_children_record;
int or_thin_children(or_store *s, int is_photon, int64_t max_per_parent, uint64_t seed,
                     int64_t step, or_thin_children_record *rec);

/* Non-perturbative (Schwinger) pairs of Sec. V.B on a periodic Yee grid (f->kind ==
 * OR_FIELD_YEE), one global step n = step of length dt.  The field of cell (i, j, k), the
 * box [i, i+1) x [j, j+1) x [k, k+1) in units of dx from the origin, is taken as constant:
 * each E component is the mean of its four staggered samples on the cell (Ex at (i+1/2,
 * j..j+1, k..k+1), Ey at (i..i+1, j+1/2, k..k+1), Ez at (i..i+1, j..j+1, k+1/2)); the
 * magnetic field is neglected.  With e = |E| eps_r = E / E_S the probability of a pair in
 * the cell during the step is P = R_S V dt, R_S = e^2 exp(-pi / e) / (4 pi^3 eps_r^4) (the
 * reduced Compton length is eps_r in units of c / omega), V = dx0 dx1 dx2.  The cells are
 * visited in index order c = i + n0 (j + n1 k); cell c creates a pair iff u < P, u the first
 * two words of the Philox draw keyed by c with counter (step, 7 << 16, seed lo, seed hi);
 * the pair sits at origin + (i + u_x, j + u_y, k + u_z) dx, u_x..u_z = (w_m + 1/2) 2^-32 from
 * the first three words of the draw with purpose 8; both have zero momentum, weight
 * `weight`, no parent, birth ((step + 1) << 14), ids or_child_id(c, seed, step, 0, 9) and
 * (..., 10).  Returns 0. */
typedef struct {
  int64_t cells;      /* cells visited */
  int64_t pairs;      /* pairs created (dropped ones included) */
  int64_t dropped;    /* leptons beyond a store's capacity */
  int64_t saturated;  /* cells with P >= 1 (at most one pair per cell and step) */
  double expected;    /* sum of min(P, 1) over the cells */
} or_schwinger_record;
int or_schwinger(or_store *st /* [3] */, const or_field *f, double dt, double eps_r,
                 double weight, uint64_t seed, int64_t step, or_schwinger_record *rec);

/* Batch helpers for statistical pins: run the generators on Philox draws keyed by `key`. */
int64_t or_emission_trials(const or_tables *t, int backend, double chi, double gamma, double dtfac,
                           uint64_t key, int64_t n, double *delta_out);
int64_t or_pair_trials(const or_tables *t, int backend, double chi_g, double kabs, double dtfac,
                       uint64_t key, int64_t n, double *delta_out);

/* The emission event generators of Sec. IV.G, as independent trials for one lepton state
 * (chi, gamma) over one interval of rate prefactor dtfac: trial first + i (i < n) draws
 * (r1, r2) from Philox, counter (trial, trial >> 32, 0, 0) and key, and writes the emitted
 * photon's delta to delta_out[i], or 0 when it emits nothing.
 *   OR_GEN_MODIFIED     Eq. (25): delta = r1^3, emission iff r2 < P_m(r1)
 *   OR_GEN_ALTERNATIVE  Eq. (24): delta = r1, emission iff r2 < P(r1)
 *   OR_GEN_STANDARD     Eqs. (22)-(23): emission iff r1 < W(1), delta the root of
 *                       W(delta) = r2 W(1), W(x) = int_{delta_min}^{x} P(delta) d delta
 * Returns the number of emissions, or -1 for an unknown generator or, for the standard
 * one, delta_min outside (0, 1). */
#define OR_GEN_MODIFIED 0
#define OR_GEN_ALTERNATIVE 1
#define OR_GEN_STANDARD 2
int64_t or_generator_trials(const or_tables *t, int backend, int generator, double chi,
                            double gamma, double dtfac, double delta_min, uint64_t key,
                            int64_t first, int64_t n, double *delta_out);
/* W(x) of the standard generator (Eq. (23)), for x in [delta_min, 1]. */
double or_standard_w(const or_tables *t, int backend, double chi, double gamma, double dtfac,
                     double delta_min, double x);

#ifdef __cplusplus
}
#endif
#endif

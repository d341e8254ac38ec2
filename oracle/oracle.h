/*
 * Reference oracle for operator-split stochastic reaction-diffusion on
 * tetrahedral meshes (Hepburn, Chen & De Schutter, "Accurate
 * Reaction-Diffusion Operator Splitting on Tetrahedral Meshes for Parallel
 * Stochastic Molecular Simulations", arXiv:1512.03126).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation of Algorithm 1 of the paper, used to check the GPU library.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no source with the GPU library: its
 * geometry, Philox generator, logarithm, binomial sampler, SSA and split are
 * written here from the paper and from the published definitions they name.
 *
 * Every call is single-threaded; no function retains a caller pointer.
 */
#ifndef RDOS_ORACLE_H
#define RDOS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_sim orc_sim;

/* Mesh + model in one call.
 *   xyz        [n_verts][3] vertex coordinates, metres
 *   tet_verts  [n_tets][4]  vertex ids of each tetrahedron
 *   D          [n_species]  diffusion coefficients, m^2/s (0 = immobile)
 *   reaction r: reac_n[r] in 0..2 reactants reac_ids[r][0..1],
 *               prod_n[r] in 0..3 products  prod_ids[r][0..2],
 *               rate k[r] in SI (0th order M/s, 1st 1/s, 2nd 1/(M s))
 *   tau_scale  in (0,1]: shortens tau below the paper's upper limit
 * Returns NULL and writes a message to err (if non-NULL, >= 256 bytes) on
 * invalid input (degenerate tet, face shared by three tets, bad ids, no
 * diffusing species). */
orc_sim *orc_create(int32_t n_verts, const double *xyz, int32_t n_tets,
                    const int32_t *tet_verts, int32_t n_species,
                    const double *D, int32_t n_reac, const int32_t *reac_n,
                    const int32_t *reac_ids, const int32_t *prod_n,
                    const int32_t *prod_ids, const double *k,
                    double tau_scale, uint64_t seed, int32_t realization,
                    char *err);
/* The same for a surface of triangles (surface diffusion, Sec. III.A):
 * tri_verts[n_tris][3]; edge e is opposite local vertex e and slot 3 is a
 * boundary.  r_e = L_e / (A delta_e), the unit of amount is N_A A with A in
 * m^2, so rates are k in mol/(m^2 s) (0th order), 1/s (1st), m^2/(mol s)
 * (2nd).  Errors as above (degenerate triangle, edge on three triangles). */
orc_sim *orc_create_surface(int32_t n_verts, const double *xyz, int32_t n_tris, const int32_t *tri_verts,
                            int32_t n_species, const double *D, int32_t n_reac, const int32_t *reac_n,
                            const int32_t *reac_ids, const int32_t *prod_n, const int32_t *prod_ids,
                            const double *k, double tau_scale, uint64_t seed, int32_t realization, char *err);
void orc_destroy(orc_sim *s);

double orc_tau(const orc_sim *s);
/* Ablation: 1 = "first-order" splitting (n drawn from the count at the end of
 * the period rather than the mean occupancy), the paper's Fig. 7 comparison. */
void orc_set_first_order(orc_sim *s, int on);
/* Method options: the one-by-one / multinomial-function switch point
 * (default 10), tau from the (k+1)-th smallest 1/(D g) (default k = 0;
 * returns the new tau), and a reaction restricted to a set of tets. */
void orc_set_split_threshold(orc_sim *s, int threshold);
/* Transfer form (Sec. II.B, last sentences): 0 (default) draws n =
 * binomial(SR(Nbar), zeta) and splits it over the faces; 1 splits SR(Nbar) at
 * once over the faces with weights zeta w_f and "stay" with 1 - zeta (if
 * more than the molecules present would leave, those present are split as in
 * form 0).  Same law, different draws. */
void orc_set_transfer_form(orc_sim *s, int form);
double orc_set_tau_outliers(orc_sim *s, int32_t k);
void orc_set_reaction_region(orc_sim *s, int32_t r, int32_t n, const int32_t *tets);
void orc_geometry(const orc_sim *s, int32_t *nbr /*[T][4]*/, double *w /*[T][4]*/,
                  double *g /*[T]*/, double *nav /*[T]*/, double *vol /*[T]*/,
                  double *area /*[T][4]*/);

void orc_set_counts(orc_sim *s, int32_t species, const int32_t *counts);
void orc_get_counts(const orc_sim *s, int32_t species, int32_t *counts);
void orc_set_state(orc_sim *s, int64_t step_index, double t);
void orc_get_time(const orc_sim *s, double *t, int64_t *step_index);

/* One period of Algorithm 1 of length tau_k at the current step index. When
 * nbar_out / n_out are non-NULL they receive, per [species][tet], the mean
 * occupancy and the gross number of molecules that left. */
void orc_step(orc_sim *s, double tau_k, double *nbar_out, int32_t *n_out);
void orc_run_steps(orc_sim *s, int64_t n);        /* n full periods */
void orc_run_until(orc_sim *s, double t_end);     /* Step 1 alignment */

/* Building blocks, exposed so the tests can pin them one by one. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint64_t seed, int32_t realization, uint32_t stream,
                   uint32_t tet, uint32_t step, uint32_t j);
double orc_ln(double x);
/* Binomial(n, p) from the stream (seed, realization, stream, tet, step),
 * starting at draw index *j; *j is advanced past the draws used. */
int64_t orc_binomial(int64_t n, double p, uint64_t seed, int32_t realization,
                     uint32_t stream, uint32_t tet, uint32_t step, uint32_t *j);
/* Multinomial split of n over weights w[0..3] (nbr[f] < 0 = no neighbour) as
 * in the diffusion step; writes out[4]; returns the final draw index. */
uint32_t orc_split(int64_t n, const double *w, const int32_t *nbr,
                   uint64_t seed, int32_t realization, uint32_t stream,
                   uint32_t tet, uint32_t step, uint32_t j, int64_t *out);

/* Batch helpers for statistical tests: sample i uses stream 0, tet i, step 0. */
void orc_binomial_many(int64_t n, double p, uint64_t seed, int32_t count, int64_t *out);
void orc_split_many(int64_t n, const double *w, const int32_t *nbr, uint64_t seed,
                    int32_t count, int64_t *out /*[count][4]*/);
/* count samples of the form-1 split of n molecules with zeta, out[count][4] */
void orc_split_scaled_many(int64_t n, double zeta, const double *w, const int32_t *nbr, uint64_t seed,
                           int32_t count, int32_t threshold, int64_t *out);
void orc_split_many_threshold(int64_t n, const double *w, const int32_t *nbr, uint64_t seed,
                              int32_t count, int32_t threshold, int64_t *out /*[count][4]*/);

#ifdef __cplusplus
}
#endif
#endif

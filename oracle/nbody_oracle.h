/*
 * nbody_oracle.h -- CPU reference of the gravitational octree method.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library under paper_1811_02761_amd/) never calls it and shares no code
 * with it.
 *
 * What it computes (Miki, "Gravitational octree code performance evaluation
 * on Volta GPU", CPC 2019):
 *   - Eq. 1 (Sec. 1): softened Newtonian acceleration by direct summation, FP64.
 *   - The tree method of Sec. 1 step by step: Morton keys of a power-of-two
 *     root cube, a stable key sort, a level-order octree whose leaves hold at
 *     most leaf_max particles, monopole moments (mass and centre of mass,
 *     "calcNode", Sec. 2.2), i-groups sharing one interaction list, the
 *     acceleration MAC of Eq. 2 evaluated once per (group, cell), and the sum
 *     of Eq. 1 over the accepted pseudo-particles and opened leaf particles.
 *   - Leapfrog (kick-drift-kick) integration.
 *   - A small MLP (forward, analytic backward) used as a cost model.
 *
 * Conventions: arrays are plain C arrays owned by the caller; "sorted" arrays
 * are indexed by position in key order; every function is synchronous.
 * Floating-point expressions in FP32 are written operation by operation and
 * the library is compiled with -ffp-contract=off; fmaf is used exactly where
 * the definition names a fused multiply-add.
 */
#ifndef NBODY_ORACLE_H
#define NBODY_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Eq. 1 in FP64 for the target particles `tgt` (NULL: all n). Inputs are
 * FP64. j == i is skipped. Outputs per target: acceleration, the L1 scale
 * A_i = sum_j G m_j |r_ij| / (r_ij^2+eps^2)^(3/2) (may be NULL) and the
 * potential phi_i = -sum_{j!=i} G m_j / sqrt(r_ij^2+eps^2) (may be NULL). */
void orc_direct(int64_t n, const double *x, const double *y, const double *z,
                const double *m, int64_t nt, const int64_t *tgt, double G,
                double eps, double *ax, double *ay, double *az, double *aabs,
                double *phi, int nthreads);

/* Root cube: lo = exact FP32 minimum per axis; ext = max over axes of
 * (double)max - (double)min; L = smallest power of two >= ext (1 if ext==0).
 * box[0..2] = lo (as double), box[3] = L. Returns 0, or -1 if any
 * coordinate is not finite. */
int orc_root_cube(int64_t n, const float *x, const float *y, const float *z,
                  double box[4]);

/* 63-bit Morton keys: q_k = min(floor(((double)x_k - lo_k) * 2^21 / L),
 * 2^21-1); bit b of q_x, q_y, q_z goes to key bits 3b+2, 3b+1, 3b. */
void orc_keys(int64_t n, const float *x, const float *y, const float *z,
              const double box[4], uint64_t *keys);

/* The same with `bits` bits per axis (3 * bits key bits). */
void orc_keys_bits(int64_t n, const float *x, const float *y, const float *z,
                   const double box[4], int32_t bits, uint64_t *keys);

/* Stable ascending sort by key: perm[s] = original index of the particle
 * at sorted position s; keys_sorted[s] = keys[perm[s]]. */
void orc_sort(int64_t n, const uint64_t *keys, int64_t *perm,
              uint64_t *keys_sorted);

/* Level-order octree of sorted keys. A cell at level l covers the particles
 * whose key >> 3(21-l) equals its prefix; it is split iff (it holds more
 * than leaf_max particles or l < min_level) and l < 21; only non-empty
 * octants become children,
 * stored consecutively in octant order. Cells are numbered by level, then by
 * prefix. Returns the number of cells; if it exceeds cap, nothing beyond cap
 * is written (call with cap = 0 to query). first_child = -1 and n_child = 0
 * for leaves; parent = -1 for the root. */
int64_t orc_build(int64_t n, const uint64_t *keys_sorted, int32_t leaf_max,
                  int32_t min_level, int64_t cap, int32_t *level, int64_t *pbegin,
                  int64_t *pcount, int64_t *first_child, int32_t *n_child,
                  int64_t *parent);

/* Monopole moments of every cell. M and S = sum m x are FP64: sequential in
 * sorted order for a leaf, the children's unrounded sums in octant order for
 * an internal cell. Stored: m32 = (float)M; com = (float)(S/M) (the first
 * member's position if M == 0); b2 = max over members of
 * fmaf(dz,dz,fmaf(dy,dy,dx*dx)) with d = x_i - com in FP32; q = (G*m32)*b2
 * in FP32. Particle arrays are sorted FP32. Dm/Dsx/Dsy/Dsz may be NULL. */
void orc_moments(int64_t ncell, const int64_t *pbegin, const int64_t *pcount,
                 const int64_t *first_child, const int32_t *n_child,
                 const float *sx, const float *sy, const float *sz,
                 const float *sm, float G, float *m32, float *comx,
                 float *comy, float *comz, float *b2, float *q, double *Dm,
                 double *Dsx, double *Dsy, double *Dsz);

/* i-groups: cells at min_level or deeper holding at most group_max
 * particles (or leaves) whose parent is not such a cell; the root if n <=
 * group_max and min_level == 0. Listed in sorted-particle order; a group cell holding more than
 * group_max particles is cut into consecutive pieces of group_max. With
 * merge != 0, consecutive sibling group cells are joined greedily (in octant
 * order) while the joined count stays within group_max. Returns the count
 * (query with cap = 0). gcell = the group's cell (the parent for a joined
 * group). */
int64_t orc_groups(int64_t ncell, const int32_t *level, const int64_t *pbegin,
                   const int64_t *pcount, const int64_t *first_child,
                   const int32_t *n_child, int32_t group_max, int32_t merge,
                   int32_t min_level, int64_t cap, int64_t *gbegin, int64_t *gcount,
                   int64_t *gcell);

/* Per group: exact FP32 bounding box of the members, amin = min over members
 * of sqrtf(fmaf(az,az,fmaf(ay,ay,ax*ax))) of the previous acceleration, and
 * dA = delta_acc * amin (FP32). With a_old == NULL, amin = dA = 0. */
void orc_group_bounds(int64_t ngroup, const int64_t *gbegin,
                      const int64_t *gcount, const float *sx, const float *sy,
                      const float *sz, const float *sax, const float *say,
                      const float *saz, float delta_acc, float *lo3, float *hi3,
                      float *amin, float *dA);

/* Eq. 2 for one (group, cell) pair, multiplied through by d^4 > 0:
 * accept iff d2 > b2 and dA * (d2*d2) >= q, where d2 is the squared distance
 * from the cell's centre of mass to the group's box. With bootstrap != 0 the
 * geometric criterion d2 > 4 b2 is used instead (no previous acceleration). */
int orc_mac(const float lo[3], const float hi[3], float dA, int bootstrap,
            float cx, float cy, float cz, float b2, float q);

/* Group-wise walk: for each group, collect the accepted cells (as
 * pseudo-particles com, m32) and the particles of opened leaves, then sum
 * Eq. 1 over them in FP64 for every member. Outputs (sorted order) FP64
 * accelerations; when phi is not NULL the potential over the same entries,
 * phi_i = -sum G m_j / sqrt(r_ij^2 + eps^2) with the particle's own entry
 * left out; per group the number of entries and an order-independent
 * hash of the entry identities (cell c -> c, leaf particle s -> 2^40 + s).
 * groot (may be NULL: the root, cell 0) gives each group's starting cell. */
void orc_walk(int64_t n, const float *sx, const float *sy, const float *sz,
              const float *sm, int64_t ncell, const int64_t *pbegin,
              const int64_t *pcount, const int64_t *first_child,
              const int32_t *n_child, const float *m32, const float *comx,
              const float *comy, const float *comz, const float *b2,
              const float *q, int64_t ngroup, const int64_t *gbegin,
              const int64_t *gcount, const float *glo3, const float *ghi3,
              const float *gdA, const int64_t *groot, int bootstrap, double G,
              double eps, double *ax, double *ay, double *az, double *phi,
              int64_t *gentries, uint64_t *ghash, int nthreads);

/* Entry-identity mixer used by the per-group hash (splitmix64 finaliser). */
uint64_t orc_mix64(uint64_t v);

/* MLP cost model 4 -> H -> H -> 1 with tanh hidden units, FP64.
 * Weight layout (row-major, output-major): mu[4] is[4] W1[H][4] b1[H]
 * W2[H][H] b2[H] W3[H] b3. The inputs are first standardised, z = (f - mu)
 * * is (fixed constants of the model, set from the training data). Forward:
 * y = W3 h2 + b3. Loss over a batch: mean (y - t)^2.
 * orc_mlp_grad returns the loss and the gradient (same layout). */
int64_t orc_mlp_nparams(int32_t hidden);
void orc_mlp_forward(int32_t hidden, const double *w, int64_t rows,
                     const double *feat, double *y);
double orc_mlp_grad(int32_t hidden, const double *w, int64_t rows,
                    const double *feat, const double *target, double *grad);

#ifdef __cplusplus
}
#endif
#endif

/*
 * bispec.h -- C ABI of the MI355X (gfx950) FFT-based binned bispectrum estimator.
 *
 * The estimator (Shaw et al., "A fast estimator for quantifying the shape
 * dependence of the 3D bispectrum", arXiv:2107.14564, Section 2) takes a real
 * field delta(x) on a periodic N_g^3 grid in a cube of side L and returns, for
 * every selected triangle bin (a1 >= a2 >= a3) of spherical k-shells,
 *
 *     B(a1,a2,a3) = [V N_tri N_g^3]^-1 sum_x D_a1(x) D_a2(x) D_a3(x)     (eq. bsfin)
 *     D_n(x)      = sum_{k in shell n} Z(k) Delta(k) e^{ik.x}             (eq. iFT)
 *     N_tri       = N_g^-3 sum_x I_a1(x) I_a2(x) I_a3(x)                  (eq. Ntri2)
 *     I_n(x)      = sum_{k in shell n} e^{ik.x}                           (eq. 2FT)
 *
 * which equals the direct closed-triangle sum of eq. binbs exactly while every
 * mode satisfies k < 2 pi N_g / (3 L) (Section 2.2, eq. 3FT).  Here
 * Delta(k) = dV sum_x delta(x) e^{-ik.x} (the convention under which eq. bs reads
 * <Delta Delta Delta> = V B), V = L^3, dV = V / N_g^3, and Z(k) = 1 + beta (k_z/|k|)^2
 * is the optional linear redshift-space factor of eq. RSD (line of sight = z).
 * Bins are labelled (k1, mu, t) by eq. shape from the shells' mean |k|.
 *
 * Conventions shared by every entry point
 *   - k = k_f m, k_f = 2 pi / L, m integer.  Shells have width dk = w k_f with
 *     w >= 1 (Section 2.1: widths below one grid spacing are not meaningful);
 *     shell n (1..n_shells) holds the modes with (n - 1/2) w <= |m| < (n + 1/2) w,
 *     decided exactly on the integer |m|^2 as
 *         (2n-1)^2 w^2 <= 4 |m|^2 < (2n+1)^2 w^2   (evaluated in IEEE double).
 *   - A bin is closable when a2 + a3 >= a1; only closable bins are selected.
 *   - Every used mode must lie below the aliasing cutoff: (n_shells + 1/2) w <= N_g/3,
 *     else BISPEC_ECUTOFF.
 *   - The shell fields and the triple sums live on estimator grids of G <= N_g
 *     points per side: Section 2.2's aliasing argument applied to G shows that
 *     the G^3-point sums of eqs. bsfin and Ntri2 (with N_g^3 replaced by G^3)
 *     pick exactly the closed triangles of a bin (a1, a2, a3) once
 *     G > R_a1 + R_a2 + R_a3 (R_n the largest mode component of shell n; and
 *     G > 2 R_a1, so a shell's modes keep their signed frequencies), so B and
 *     N_tri do not depend on G.  A plan splits its triangles into grid
 *     classes, each on the smallest grid that is exact for all of its
 *     triangles and worth its extra shell transforms (a cost model);
 *     bispec_grid_classes tells the split.  The largest grid, the plan's
 *     estimator grid (bispec_estimator_grid), is the smallest supported size
 *     above 3 max|m_i| unless n_est forces one grid.  Only the forward
 *     transform (and the last inverse of bispec_grad) runs at N_g.
 *   - delta is float32 [N_g][N_g][N_g], z fastest (C order), on the device.
 *   - B is float64 [n_tri] on the device, ordered like bispec_triangles().
 *
 * Threading / streams: calls on different plans may run concurrently; calls on
 * one plan must be serialised by the caller.  bispec_run and bispec_grad are
 * asynchronous on the given HIP stream and allocate nothing; only bispec_plan
 * allocates device memory and synchronises.
 *
 * Errors: every call returns BISPEC_OK (0) or a negative status and never
 * throws; bispec_last_error() returns the calling thread's last message.
 */
#ifndef BISPEC_H
#define BISPEC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bispec_plan_s* bispec_plan_t;
typedef struct bispec_many_s* bispec_many_t;

enum bispec_status {
  BISPEC_OK = 0,
  BISPEC_EINVAL = -1,   /* bad argument or configuration                         */
  BISPEC_ECUTOFF = -2,  /* a shell reaches k >= 2 pi N_g / (3 L) (eq. 3FT)        */
  BISPEC_ENOMEM = -3,   /* workspace exceeds free device memory or BISPEC_MAX_BYTES */
  BISPEC_EHIP = -4,     /* HIP runtime error (message holds hipGetErrorString)    */
  BISPEC_ESTATE = -5,   /* call out of order (e.g. grad before any run)           */
  BISPEC_EPREC = -6     /* an N_tri sum was not within 1e-3 of an integer         */
};

/* Triangle selection rules. */
enum bispec_tri_mode {
  BISPEC_TRI_ALL = 0,      /* every closable shell triple                               */
  BISPEC_TRI_K1SET = 1,    /* closable triples with a1 in k1_shells[0..n_k1)            */
  BISPEC_TRI_MUT_GRID = 2, /* per a1 in k1_shells, the triples nearest a (mu,t) grid:   */
                           /*   mu_g, t_g = linspace(0.5,1,n_mu) x linspace(0.5,1,n_t), */
                           /*   t_g mu_g >= 0.5 - 1e-12 (eq. cond),                     */
                           /*   a2 = clamp(floor(t_g a1 + 1/2), 1, a1),                 */
                           /*   a3 = clamp(floor(a1 sqrt(1 + t_g^2 - 2 mu_g t_g) + 1/2), 1, a2); */
                           /*   unique closable triples kept                            */
  BISPEC_TRI_LIST = 3      /* the n_list rows (a1,a2,a3) of list (each closable, distinct) */
};

/* Arithmetic of the triple contraction (step c); FFTs are float32 in both. */
enum bispec_precision {
  BISPEC_PREC_SPLITBF16 = 0, /* bf16 MFMA on hi+lo split operands, fp32 accumulate  */
  BISPEC_PREC_FP32 = 1       /* plain fp32 vector FMAs                               */
};

enum bispec_flags {
  BISPEC_FLAG_GRAD = 1u,         /* allocate the workspace for bispec_grad            */
  BISPEC_FLAG_STAGE_TIMING = 2u, /* record HIP events around each stage of run       */
  BISPEC_FLAG_AUTOTUNE = 4u,     /* per grid class, time the split-bf16 contraction   */
                                 /* at plan time for column-tile windows {8, 4} x     */
                                 /* 64..512 voxel ranges on pseudo-random fields and  */
                                 /* keep the fastest; with BISPEC_TUNE_CACHE naming a */
                                 /* file, choices are read from and appended to it    */
                                 /* (JSON lines keyed by a hash of the class)         */
  BISPEC_FLAG_NO_WORKSPACE = 8u, /* keep no run workspace: the plan holds its tables */
                                 /* and N_tri only and is run by bispec_run_noalloc   */
                                 /* (excludes GRAD and AUTOTUNE; not in a batch)      */
  BISPEC_FLAG_ONE_GRID = 16u     /* one grid class: every shell and triangle on the   */
                                 /* estimator grid (as a nonzero n_est does)          */
};

typedef struct bispec_config {
  int32_t n_g;            /* grid points per side: 2^a, 3*2^a or 5*2^a, 2^a >= 8, <= 1024 */
  int32_t n_shells;       /* shells 1..n_shells                                     */
  double box_l;           /* box side L (> 0); k in units of 1/L's unit             */
  double dk;              /* shell width w in units of k_f (w >= 1)                  */
  double rsd_beta;        /* linear RSD beta (0 = none), line of sight z            */
  int32_t tri_mode;       /* enum bispec_tri_mode                                   */
  int32_t n_k1;           /* K1SET / MUT_GRID: number of a1 shells                  */
  const int32_t* k1_shells; /* host array [n_k1], read only during the call        */
  int32_t n_mu, n_t;      /* MUT_GRID grid sizes (>= 2)                              */
  int64_t n_list;         /* LIST: number of rows                                   */
  const int32_t* list;    /* LIST: host array [n_list][3] (a1,a2,a3), a1>=a2>=a3>=1 */
  int32_t precision;      /* enum bispec_precision                                  */
  uint32_t flags;         /* enum bispec_flags                                      */
  int32_t n_est;          /* estimator grid G for the shell fields and triple sums:  */
                          /*   0 = grid classes up to the smallest supported size   */
                          /*   above 3 max|m_i|; else one class on this supported   */
                          /*   size, 3 max|m_i| < n_est <= n_g                      */
  int32_t order;          /* 0 or 3: the bispectrum; 4: the fourth-order           */
                          /*   polyspectrum (Section 4): bins of four shells       */
                          /*   a1 >= a2 >= a3 >= a4 with a2 + a3 + a4 >= a1,        */
                          /*   T = sum_x D D D D / (V N_quad N_g^3), N_quad =       */
                          /*   N_g^-3 sum_x I I I I; cutoff (n_s + 1/2) w <= N_g/4; */
                          /*   one grid G > 4 max|m_i|; selection ALL, K1SET or     */
                          /*   LIST (rows of 4); split-bf16 only; no GRAD,          */
                          /*   NO_WORKSPACE or batch                                */
  int32_t ell;            /* Legendre multipole of the redshift-space bispectrum   */
                          /*   (Section 3.1, line of sight z), 0, 2 or 4: every    */
                          /*   closed triangle weighted by L_ell(mu_1), mu_1 =     */
                          /*   k1_z/|k1| of its first side (shell a1), and B times */
                          /*   (2 ell + 1); 0 = the bispectrum itself.  ell > 0:  */
                          /*   order 3, no GRAD; a grid class with more than 64    */
                          /*   shells (split-bf16) or 128 (fp32) is refused        */
} bispec_config;

/* ---- host-only queries (no GPU needed) ------------------------------------ */

/* Selected triangles for cfg, ordered by (a1,a2,a3) ascending.  Writes n_tri;
 * if abc (host, [capacity][3]) and/or k1_mu_t (host, [capacity][3]: k1 in 1/L
 * units of k, mu, t from eq. shape) are non-null, fills min(n_tri, capacity)
 * rows.  Errors: EINVAL, ECUTOFF. */
int bispec_query_triangles(const bispec_config* cfg, int64_t* n_tri, int32_t* abc,
                           double* k1_mu_t, int64_t capacity);

/* Selected quadruples of an order-4 cfg (as bispec_query_triangles, four
 * columns: abcd host int32 [capacity][4]).  Errors: EINVAL, ECUTOFF. */
int bispec_query_quads(const bispec_config* cfg, int64_t* n_quad, int32_t* abcd, int64_t capacity);

/* Per-shell mode counts (host int64 [n_shells], both halves of k-space) and
 * mean |k| (host double [n_shells], in k units), Section 2.1's k_n. */
int bispec_shell_stats(const bispec_config* cfg, int64_t* counts, double* mean_k);

/* The estimator grid G that a plan of cfg would use (see n_est). */
int bispec_estimator_grid(const bispec_config* cfg, int32_t* n_est);

/* The plan's estimator-grid classes for cfg (host only): *n_classes receives
 * their number; for k < capacity, grid[k] is class k's grid and its shell
 * fields cover shells shell_lo[k] .. shell_hi[k] (1-based, inclusive); if
 * tri_class (host int32 [n_tri]) is non-null it receives each selected
 * triangle's class (triangles ordered as bispec_query_triangles).  Classes are
 * ordered by grid, ascending.  Any output may be null.  Errors: EINVAL, ECUTOFF. */
int bispec_grid_classes(const bispec_config* cfg, int32_t* n_classes, int32_t* grid, int32_t* shell_lo,
                        int32_t* shell_hi, int32_t capacity, int32_t* tri_class);

/* The split-bf16 contraction's work decomposition for cfg (host only, for
 * tests and tuning): for each selected triangle t < capacity, tile[t] receives
 * the index of the 16 x 16 accumulator tile that sums it (unique across the
 * plan's grid classes) and shape[t] = 16 NT + NRB of the wavefront slot that
 * owns the tile (NT column tiles, NRB row blocks: the kernel's code variant).
 * Either output may be null.  Errors: EINVAL, ECUTOFF. */
int bispec_contraction_tiles(const bispec_config* cfg, int64_t capacity, int32_t* tile, int32_t* shape);

/* Device bytes the plan keeps (run_bytes) and its peak during planning
 * (plan_peak_bytes, which includes the float64 unit shells). */
int bispec_workspace_bytes(const bispec_config* cfg, int64_t* run_bytes, int64_t* plan_peak_bytes);

/* ---- plan / run ------------------------------------------------------------ */

/* Validate cfg, build shell and triangle tables, allocate the workspace on the
 * current device, compute N_tri on the GPU in float64 from the unit shells
 * (eqs. 2FT, Ntri2), round and check them (EPREC), then free the unit shells.
 * hip_stream: a hipStream_t (null = default stream); the call synchronises it.
 * *out receives the plan (owned by the caller; release with bispec_destroy).
 * Voxel-slab streaming: when the plan with whole shell fields resident does
 * not fit (hipMemGetInfo, BISPEC_MAX_BYTES), the number of x-slabs per grid
 * class is doubled until it does (at least the env var BISPEC_SLABS, default
 * 1): the fields, second-pass intermediates and partial sums then hold one
 * slab of x-planes, every run computes a class's x pass once and, slab by
 * slab, its y and z passes and the slab's triple sums, added into B in slab
 * order (the same for N_tri at plan time).  Not for order 4 or GRAD plans;
 * bispec_copy_field of a streamed plan is ESTATE; its stage times put the
 * contraction in the shell-pass stage.
 * Errors: EINVAL, ECUTOFF, ENOMEM (checked before any allocation against
 * hipMemGetInfo and the env var BISPEC_MAX_BYTES), EHIP, EPREC. */
int bispec_plan(const bispec_config* cfg, void* hip_stream, bispec_plan_t* out);

/* x-slabs per grid class of a plan (1: whole fields resident). */
int bispec_plan_slabs(bispec_plan_t plan, int32_t* slabs);

int bispec_num_triangles(bispec_plan_t plan, int64_t* n_tri);

/* Host copies of the plan's triangles: abc [n_tri][3] int32, k1_mu_t [n_tri][3]
 * double, ntri [n_tri] int64 (the exact triangle counts).  Any may be null. */
int bispec_triangles(bispec_plan_t plan, int32_t* abc, double* k1_mu_t, int64_t* ntri);

/* One pass of the estimator: forward R2C FFT of delta (a), per-shell masked
 * inverse FFTs to the data shells D_n (b), the triple contraction (c) and the
 * float64 normalisation B = T / (V N_tri N_g^3) (d).
 * delta: device float32 [N_g^3]; B: device float64 [n_tri].  Both caller-owned,
 * must not alias the plan's memory.  Asynchronous on hip_stream. */
int bispec_run(bispec_plan_t plan, const float* delta, double* B, void* hip_stream);
/* (ESTATE for a plan made with BISPEC_FLAG_NO_WORKSPACE.) */

/* bispec_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same pass, with every run buffer (spectrum, shell-pass intermediates, shell
 * fields, contraction partials) placed in a static per-device scratch array of
 * 256 MiB instead of the plan's workspace.  Calls no allocating routine; the
 * caller passes delta and B as for bispec_run.  Works with any plan whose run
 * buffers fit (e.g. N_g <= 64 with 20 shells), including plans made with
 * BISPEC_FLAG_NO_WORKSPACE, which hold no workspace of their own.
 * Every call on a device shares that device's scratch and clears the part it
 * uses first (one fill kernel on hip_stream), so calls that overlap on
 * one device race and must be serialised by the caller.  bispec_grad and
 * bispec_copy_field keep referring to the last bispec_run, not to this call.
 * The plan's device must be current.
 * Errors: EINVAL (null argument, run buffers beyond 256 MiB, plan of another
 * device), EHIP. */
int bispec_run_noalloc(bispec_plan_t plan, const float* delta, double* B, void* hip_stream);

/* Vector-Jacobian product of the last bispec_run on this plan (needs
 * BISPEC_FLAG_GRAD): gdelta(x) = sum_t gB_t dB_t/d delta(x), the derivative of
 * eq. bsfin through eq. iFT: per shell n the adjoint field
 * G_n(x) = sum over the bins t with a side in shell n of
 * gB_t / (V N_tri,t N_g^3) times the product of the bin's other two fields at x,
 * then each G_n forward-transformed and restricted to the modes of shell n
 * (times Z(k) for RSD), summed, and transformed back to the grid (the adjoint
 * of eq. iFT and of the forward transform).  Split-bf16 plans build G_n on the
 * matrix cores (float32 chains, float64 sums), float32 plans on the vector ALU
 * in float64; the transforms run in float32.
 * gB: device float64 [n_tri]; gdelta: device float32 [N_g^3] (overwritten).
 * Asynchronous on hip_stream; allocates nothing (the plan holds the adjoint
 * buffers).
 * Errors: ESTATE when no run preceded or the plan lacks BISPEC_FLAG_GRAD. */
int bispec_grad(bispec_plan_t plan, const double* gB, float* gdelta, void* hip_stream);

/* Host copies of an order-4 plan's bins: abcd [n][4] int32 and nquad [n] int64
 * (the exact closed-quadruple counts); bispec_num_triangles gives n.  Either
 * may be null.  EINVAL for a bispectrum plan. */
int bispec_quads(bispec_plan_t plan, int32_t* abcd, int64_t* nquad);

/* Switch the contraction arithmetic of an existing plan (enum bispec_precision). */
int bispec_set_precision(bispec_plan_t plan, int32_t precision);

/* Stage times in ms of the last run (needs BISPEC_FLAG_STAGE_TIMING; the
 * caller synchronises the stream first): ms[0] forward FFT, ms[1] inverse
 * shell FFTs, ms[2] contraction, ms[3] normalisation.  n = entries wanted (<= 4). */
int bispec_stage_times(bispec_plan_t plan, float* ms, int32_t n);

/* The plan's grid classes as built (after autotuning): for k < capacity,
 * grid[k], the split-bf16 contraction's voxel-range count n_krange[k] (ranges
 * of work groups), column-tile window max_cols[k], work groups per range
 * n_wg[k], replicas rep[k] (a class whose tiling fits one work group with few
 * busy wavefronts runs rep copies of it on rep consecutive voxel blocks per
 * step: 1, 2, 3, 4 or 6), the autotuned time of one contraction launch of the class
 * alone tuned_ms[k] (0 if not tuned) and tune_source[k] (0 default, 1 timed at
 * plan time, 2 read from the tuning cache).  Any output array may be null. */
int bispec_plan_classes(bispec_plan_t plan, int32_t capacity, int32_t* n_classes, int32_t* grid, int32_t* n_krange,
                        int32_t* max_cols, int32_t* n_wg, int32_t* rep, float* tuned_ms, int32_t* tune_source);

/* Inspection (tests): the grid on which bispec_copy_field returns shell n
 * (the largest grid of the classes whose fields cover it).  EINVAL if no
 * selected triangle uses a class covering the shell. */
int bispec_field_grid(bispec_plan_t plan, int32_t shell, int32_t* grid);

/* Inspection (tests): copy the data shell D_n of the last run on the grid of
 * bispec_field_grid, divided by dV N_g^{3/2} (the plan's internal scale), into
 * dst (device float32 [g^3], C order). */
int bispec_copy_field(bispec_plan_t plan, int32_t shell, float* dst, void* hip_stream);

/* Inspection (tests): as bispec_copy_field, from grid class cls (0-based, in
 * the order of bispec_grid_classes), whose fields cover shell; dst is device
 * float32 [g^3] with g that class's grid. */
int bispec_copy_class_field(bispec_plan_t plan, int32_t cls, int32_t shell, float* dst, void* hip_stream);

/* Release a plan (not one obtained from bispec_many_plan: EINVAL). */
int bispec_destroy(bispec_plan_t plan);

/* ---- batched form: many realisations / configurations ---------------------- */
/* The same estimator over n configurations (any mix of n_g, shells, selection,
 * precision; no BISPEC_FLAG_GRAD), e.g. an ensemble of realisations as in the
 * validation of Section 3.  One shared run workspace sized for the largest
 * member; tables and N_tri per member; identical consecutive members run as
 * cohorts (bispec_many_units).  hip_stream as for bispec_plan.
 * Errors: as bispec_plan, plus EINVAL for n < 1 or a GRAD flag. */
int bispec_plan_many(const bispec_config* cfgs, int32_t n, void* hip_stream, bispec_many_t* out);

/* Packed layout: member i reads delta[delta_off[i] .. delta_off[i+1]) (its
 * N_g^3 field, C order) and writes B[b_off[i] .. b_off[i+1]) (its n_tri
 * results, ordered as bispec_triangles of that member).  delta_off and b_off
 * are host int64 [n + 1]; n (host) receives the member count.  Any may be null. */
int bispec_many_layout(bispec_many_t batch, int32_t* n, int64_t* delta_off, int64_t* b_off);

/* Launch units of the batch: runs of identical consecutive members (same
 * configuration, split-bf16, no BISPEC_FLAG_AUTOTUNE; e.g. the realisations of
 * an ensemble) form cohorts whose forward transforms and shell passes run as
 * one launch per pass for all their members (cohorts are split so their
 * per-member spectra and pass intermediates stay within 8 GiB); every other
 * member is a unit of its own.  (The contraction and the reductions of every
 * split-bf16 member run as one launch each in any case.)  n_units (host) receives the number
 * of units, n_cohort_members (may be null) the number of members in cohorts. */
int bispec_many_units(bispec_many_t batch, int32_t* n_units, int32_t* n_cohort_members);

/* Member i as a plan handle for bispec_num_triangles / bispec_triangles /
 * bispec_stage_times queries (owned by the batch: never bispec_destroy it). */
int bispec_many_plan(bispec_many_t batch, int32_t i, bispec_plan_t* plan);

/* All members, back to back, asynchronously on hip_stream.  delta: device
 * float32 packed fields; B: device float64 packed results (caller-owned).
 * use_graph != 0: the launches of all members are captured once into a HIP
 * graph (on a private stream; recaptured when delta or B change) and replayed
 * with one hipGraphLaunch on hip_stream; 0: launched directly. */
int bispec_run_many(bispec_many_t batch, const float* delta, double* B, int32_t use_graph, void* hip_stream);

int bispec_destroy_many(bispec_many_t batch);

/* Last error message of the calling thread ("" if none). */
const char* bispec_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BISPEC_H */

/*
 * libvie — block-preconditioned VIE-FFT solver on one AMD Instinct MI355X.
 *
 * Solves the volume integral equation of Huang & Sha, "A Parallel Block
 * Preconditioner Based VIE-FFT Algorithm for Modeling Electromagnetic
 * Response from Nanostructures" (arXiv 2501.13512), Sec. II:
 *
 *   eq. (2)  E_tot = J / (j omega (eps - eps0))
 *   eq. (3)  E_tot = E_inc + E_s,   E_s from eq. (1) with the dyadic
 *            Green's function G = (I + grad grad / k0^2) g,
 *            g = exp(-j k0 R) / (4 pi R)   (exp(+j omega t) convention)
 *   eq. (4)  the resulting equation for J, discretised on a uniform voxel
 *            grid into the 3x3-block system A x = b of eq. (6).
 *
 * The library works with P = J / (j omega eps0) (same Krylov iterates as J
 * up to a constant), so with chi = eps_r - 1 and S = non-vacuum voxels:
 *   (A P)_m = P_m / chi_m - sum_{n in S} T(m - n) P_n = E_inc(r_m),  m in S,
 * T(m) = k0^2 dV G(r_m - r_0) for m != 0 (voxel-centre sampling), and for
 * m = 0 the integral of k0^2 G over the sphere of the voxel's volume.  The
 * product A x is the paper's FFT acceleration (Sec. I: Toeplitz structure of
 * the uniform grid, zero-padded 3-D FFT).  The system is solved by BiCGSTAB
 * (Sec. II-B) with the block-diagonal right preconditioner of eq. (10): the
 * scatterer is partitioned into blocks, each block matrix A_k (all x/y/z
 * couplings, eq. (11)) is solved by an inner BiCGSTAB-FFT to a loose
 * tolerance, and the block solutions are merged into one vector.
 *
 * Conventions
 *  - Fields and currents are complex double, interleaved (re, im), stored
 *    component-major [3][nz][ny][nx] with x fastest (same bytes as
 *    C99 double _Complex and torch.complex128).
 *  - Voxel (i, j, k) has its centre at ((i+1/2)dx, (j+1/2)dy, (k+1/2)dz)
 *    from the grid corner; phases are referred to the grid centre.
 *  - eps_r == 1 (exactly) marks vacuum: no unknown there, outputs are 0.
 *  - Lossy media have Im(eps_r) < 0 (exp(+j omega t)).
 *  - Length units are arbitrary but common to spacing and wavelength;
 *    k0 = 2 pi / wavelength.
 *  - Grid sizes: 1 <= n <= 256 per axis (FFT lengths up to 512).
 *
 * Errors: every call returns vie_status.  0 = success, > 0 = warning with
 * results written, < 0 = error.  vie_last_error() gives a message for the
 * calling thread's last non-OK status.  No C++ exception crosses this ABI.
 *
 * Ownership: handles are created and freed by the library (matching
 * _create/_destroy).  Host arrays passed in are owned by the caller and only
 * read during the call.  Device pointers ("_dev") are borrowed for the call:
 * they must be device memory of the context's GPU, are accessed in order on
 * the given HIP stream (hipStream_t passed as void*, NULL = default stream),
 * and must stay valid until that stream reaches the end of the call's work.
 * Calls on one problem are serialised by the library; a problem holds the
 * Krylov state of one solve at a time.
 */
#ifndef VIE_H
#define VIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VIE_ABI_VERSION 15

typedef enum {
  VIE_OK = 0,
  VIE_NOT_CONVERGED = 1,   /* iteration cap reached; best iterate and stats written */
  VIE_EINVAL = -1,         /* invalid argument (sizes, non-finite values, block ids, ...) */
  VIE_ENOMEM = -2,         /* device or host allocation failed */
  VIE_EDEVICE = -3,        /* no usable HIP device, or a HIP runtime error */
  VIE_EBREAKDOWN = -4,     /* Krylov breakdown (BiCGSTAB: rho, <rhat,v> or <t,t> = 0; CGS: rho or <rhat,v> = 0;
                              GMRES: singular least-squares; or non-finite); last iterate written */
  VIE_EBUSY = -5,          /* resource budget exceeded */
  VIE_ECANCELLED = -6,
  VIE_EINTERNAL = -7,
  VIE_ETIMEDOUT = -8          /* vie_wait: not finished within the timeout (ticket still valid) */
} vie_status;

typedef struct vie_context vie_context;
typedef struct vie_problem vie_problem;
typedef struct vie_request* vie_ticket;

/* Uniform grid (Sec. II-A: hexahedral mesh, staircase geometry). */
typedef struct {
  int32_t nx, ny, nz;
  double dx, dy, dz;
  double wavelength;
} vie_grid;

typedef enum {
  VIE_FP64 = 0,   /* every product, vector and reduction in FP64 */
  VIE_MIXED = 1,  /* FFT products in complex FP32; vectors, inner products and
                     the iterative-refinement residual in FP64 */
  VIE_MIXED_INNER = 2  /* solves only: the inner block solves' products in
                          complex FP32, the full-grid products and everything
                          else in FP64 (no refinement needed); other entry
                          points taking a precision reject it */
} vie_precision;

/* Solver settings (Sec. II-B and III: outer/inner residual tolerances). */
typedef struct {
  double tol_outer;     /* stop when ||r|| / ||b|| <= tol_outer (recursive residual) */
  double tol_inner;     /* inner block solves: ||r_k|| / ||b_k|| <= tol_inner */
  int32_t maxit_outer;  /* outer BiCGSTAB steps (paper: 1000) */
  int32_t maxit_inner;  /* per inner solve */
  int32_t max_refine;   /* VIE_MIXED: iterative-refinement corrections (FP64 true residual) */
  int32_t precondition; /* 1: block-diagonal preconditioner (needs block ids), 0: none */
  int32_t precision;    /* vie_precision */
  int32_t poll_lag;     /* convergence checks trail the enqueued work by this many steps (>= 0) */
  int32_t flags;        /* VIE_FLAG_* */
  int32_t solver;       /* vie_solver */
  int32_t restart;      /* VIE_SOLVER_FGMRES: Arnoldi steps per cycle, in [1, 1000] */
} vie_opts;

/* Outer Krylov solver.  All are right preconditioned with the block
 * preconditioner of eq. (10) and start from x0 = 0.
 *  VIE_SOLVER_BICGSTAB: the BiCGSTAB of Sec. II-B; one step = two products
 *    and two preconditioner applications; maxit_outer counts steps.
 *  VIE_SOLVER_FGMRES: flexible GMRES(restart) (Saad's form for a
 *    preconditioner that varies from step to step, as the inexact inner
 *    solves make it); one Arnoldi step = one product and one preconditioner
 *    application; maxit_outer counts Arnoldi steps; stops when the minimal
 *    residual of the Arnoldi least-squares problem reaches tol_outer.
 *    Needs (2 restart + 1) vectors of 3 nx ny nz complex doubles (restart + 1
 *    without preconditioner), allocated by the first such solve of a problem
 *    and kept with it (counted in footprint_bytes; VIE_EBUSY beyond the
 *    context's budget).  Not accepted by vie_submit.
 *  VIE_SOLVER_CGS: conjugate gradient squared (Sonneveld), the other
 *    Krylov method Sec. II-B names as applicable; one step = two products
 *    and two preconditioner applications, like BiCGSTAB.  The residual is
 *    recomputed as b - A x after every step (one of the two products) and
 *    tested against tol_outer; maxit_outer counts steps.  Uses the problem's
 *    own vectors (no extra storage).  Not accepted by vie_submit. */
typedef enum {
  VIE_SOLVER_BICGSTAB = 0,
  VIE_SOLVER_FGMRES = 1,
  VIE_SOLVER_CGS = 2
} vie_solver;

/* vie_opts.flags: run the inner block iterations as individual kernel
 * launches instead of a captured HIP graph (same kernels, same results).
 * Without it, block groups whose products transform at least 2^21 points
 * per inner step (systems x 3 x padded box) are launched one by one anyway
 * (their steps outlast the host's launches, and a graph replay's start and
 * end cost more); smaller groups replay the captured step. */
#define VIE_FLAG_NO_GRAPHS 1
/* vie_opts.flags: solve every block with the batched multi-workgroup
 * kernels, also blocks small enough for the one-workgroup block solver
 * (same iteration, different summation order in the inner products). */
#define VIE_FLAG_NO_BLOCK_KERNEL 2

/* Statistics of one solve. */
typedef struct {
  int32_t outer_iters;        /* BiCGSTAB steps of the main solve */
  int32_t refine_steps;       /* VIE_MIXED correction solves */
  int32_t refine_iters;       /* BiCGSTAB steps spent in correction solves */
  int32_t final_state;        /* main loop: 1 converged, 3 breakdown, 4 iteration cap (VIE_MIXED returns
                                 VIE_OK after a cap when refinement reached tol_outer) */
  int64_t inner_iters_total;  /* sum over preconditioner applications and blocks */
  int64_t precond_applies;
  double relres_recursive;    /* ||r|| / ||b|| of the recursion at exit */
  double relres_true;         /* ||b - A x|| / ||b|| with an FP64 product */
  double seconds;             /* wall time of the call */
  int32_t* inner_hist;        /* optional (caller-owned, may be NULL): inner iteration
                                 count of every non-empty block (ascending id) for each
                                 preconditioner application, application-major */
  int64_t inner_hist_cap;     /* capacity of inner_hist in entries */
  int64_t inner_hist_len;     /* entries written */
} vie_stats;

/* Block plan summary of a problem. */
typedef struct {
  int32_t lx, ly, lz;         /* circulant FFT lengths of the full grid */
  int32_t n_blocks;           /* non-empty blocks */
  int32_t n_groups;           /* equally-shaped block batches */
  int64_t footprint_bytes;    /* device memory held by the problem */
  int32_t n_block_solver_groups;  /* groups solved one workgroup per block */
  int32_t zpass_variant[2];   /* z-pass kernel picked for the full-grid product [FP64, MIXED] */
  float zpass_tune_ms[2][5];  /* autotuner time per z-pass variant (3 runs; -1 = not timed) */
  int32_t plane_variant[2];   /* plane-kernel variant picked for the full-grid product [FP64, MIXED]
                                 (0 when its transforms are not square and small enough) */
  float plane_tune_ms[2][3];  /* autotuner time per plane variant (3 forward + inverse pairs; -1 = not timed) */
} vie_problem_info;

/* One shape group of a block plan: blocks whose bounding boxes share FFT
 * lengths, solved together (eqs. (10)-(11): every block's inner solve). */
typedef struct {
  int32_t lx, ly, lz;      /* circulant FFT lengths of the group's boxes */
  int32_t bx, by, bz;      /* the group's box (largest block bounding box) */
  int32_t n_systems;       /* blocks in the group */
  int32_t one_workgroup;   /* 1: solved by the one-workgroup block solver */
} vie_group_plan;

/* ABI version (VIE_ABI_VERSION). */
int32_t vie_abi_version(void);

/* Message for the calling thread's last non-OK status ("" if none). */
const char* vie_last_error(void);

/* Open device `device`.  hbm_budget_bytes bounds the device memory the
 * context may hold for problems (0 = no limit); problem creation beyond it
 * returns VIE_EBUSY.  Returns VIE_EDEVICE when no such HIP device exists. */
vie_status vie_context_create(int32_t device, size_t hbm_budget_bytes, vie_context** out);
/* Stops the context's server (queued requests are cancelled, running ones
 * stop after their current outer step); VIE_EBUSY, with nothing destroyed,
 * while tickets are outstanding (not yet passed to vie_wait). */
vie_status vie_context_destroy(vie_context* ctx);

/* Set up a problem (Sec. II-A and II-B): uploads 1/chi, computes (or reuses
 * from the context's cache) the Green-tensor spectra of the grid and of every
 * block shape, and allocates the Krylov state.
 *   eps_r:    nx*ny*nz complex (2 doubles each), x fastest; finite.
 *   block_id: nx*ny*nz int32 or NULL.  Voxel's block in [0, n_blocks) for
 *             non-vacuum voxels; ignored (should be -1) on vacuum voxels.
 *             Every non-vacuum voxel must have a valid id when given.
 *             Blocks partition the scatterer (eq. (10)); a block need not
 *             be a box (its product runs on its bounding box, masked).
 * VIE_EINVAL on bad sizes, non-finite values or ids out of range. */
vie_status vie_problem_create(vie_context* ctx, const vie_grid* grid, const double* eps_r, const int32_t* block_id,
                              int32_t n_blocks, vie_problem** out);

/* As vie_problem_create, with expanded blocks (the paper's future work,
 * Sec. IV): block k is solved on its voxels dilated by `overlap` voxels in
 * every axis (a (2 overlap + 1)^3 cube) within the scatterer, and only its
 * own voxels are kept from that solve (restricted additive Schwarz).  The
 * block partition still decides ownership.  overlap in [0, 256]; 0 is
 * vie_problem_create; ignored without block ids.  Larger solve sets mean
 * larger FFT boxes per block. */
vie_status vie_problem_create_overlap(vie_context* ctx, const vie_grid* grid, const double* eps_r,
                                      const int32_t* block_id, int32_t n_blocks, int32_t overlap, vie_problem** out);

/* A problem in the rooftop discretisation of Sec. II-A, eq. (5) (rooftop
 * basis functions, pulse testing; the scalar-potential and grad-div parts of
 * eqs. (7)-(9)).  The unknowns are the normal components of P on the faces
 * between cells: entry (c, z, y, x) of a 3*nx*ny*nz vector (component-major,
 * x fastest, as for voxel vectors) is the face between cell (x, y, z) and its
 * neighbour one step along axis c (x, y, z for c = 0, 1, 2).  The operator is
 *   (A P)_f = P_f / chi_f - (T P)_f,
 *   T P = k0^2 (g~ * P) + grad (g~ * div P),
 * with g~ the scalar Green's function at the cell-centre separation (its
 * mean over the sphere of the cell's volume at zero separation), * the
 * discrete convolution times the cell volume, div the cell divergence of
 * face values and grad the face gradient of cell values (both one-sided
 * differences over one cell).  The face contrast chi_f = (1 - m) / m with m
 * the mean of 1/eps_r over the face's two cells (continuity of the normal
 * flux density).  Faces between two vacuum cells carry no unknown: the
 * products and solves keep them 0.  The first and last cell layer of every
 * axis must be vacuum (VIE_EINVAL otherwise).  eps_r, block_id and n_blocks
 * as for vie_problem_create (block_id may be NULL).  Blocks (eq. (10)) are
 * sets of cells; the face between cell c and c + e_i belongs to the block of
 * c when c is a scatterer cell, else to the block of c + e_i, and block k's
 * matrix is A restricted to the faces it owns (solved on its cells'
 * bounding box grown by one cell per side).  vie_matvec,
 * vie_matvec_profile, vie_block_matvec, vie_precond_apply, vie_group_profile,
 * vie_solve and vie_solve_device (e_tot_out is then the field on every face,
 * P_f / chi_f), vie_solve_batch, vie_solve_many (a batch holds rooftop
 * problems only), vie_total_field_box (the field at every face centre of the
 * box; 0 on the faces of the last cell layer along their own axis, whose
 * second cell lies outside the grid), vie_far_field, vie_far_field_noalloc
 * and vie_rcs (each face unknown radiating from its face centre) accept it;
 * z-pass variant 1 returns VIE_EINVAL.
 * Every block group runs on the batched multi-workgroup kernels
 * (VIE_FLAG_NO_BLOCK_KERNEL has no effect). */
vie_status vie_problem_create_rooftop(vie_context* ctx, const vie_grid* grid, const double* eps_r,
                                      const int32_t* block_id, int32_t n_blocks, vie_problem** out);
vie_status vie_problem_destroy(vie_problem* p);
vie_status vie_problem_get_info(const vie_problem* p, vie_problem_info* info);

/* Pins the z-pass kernel variant (0-4; 1 = mirror columns; lengths below
 * 32 use 0 for 2-4) of every FFT product of
 * the problem in one precision, full-grid and block products alike; -1
 * restores the autotuned choice.  For kernel studies and a reproducible
 * kernel choice: the variants compute the same transform (results agree to
 * rounding; tested).  Synchronises the device; call it while no work of the
 * problem is in flight.  Errors: VIE_EINVAL for a bad precision or
 * variant. */
vie_status vie_problem_set_zpass(vie_problem* p, int32_t precision, int32_t variant);

/* Pins the plane-kernel variant of every FFT product of the problem in one
 * precision (products whose x and y lengths are equal and at most 64 run
 * the x and y transforms of a z-plane in one kernel; the variants differ in
 * the planes one workgroup takes: 0 as many as 48 KB of LDS hold, at most
 * 16; 1 at most two; 2 one); -1 restores the autotuned choice.  Same
 * transform, results agree to rounding (tested).  Synchronises the device;
 * call it while no work of the problem is in flight.  Errors: VIE_EINVAL
 * for a bad precision or variant. */
vie_status vie_problem_set_plane(vie_problem* p, int32_t precision, int32_t variant);

/* The block plan that vie_problem_create_overlap would build for these
 * inputs (same arguments and validation; overlap 0 = vie_problem_create),
 * computed on the host with no device or context: info receives the full
 * grid's FFT lengths, the non-empty block count, the shape groups, the
 * groups run by the one-workgroup solver and footprint_bytes, the device
 * memory the problem would hold with none of its spectra cached
 * (zpass_variant, zpass_tune_ms, plane_variant, plane_tune_ms all -1).  groups (optional, caller-owned)
 * receives up to groups_cap entries in the library's group order (batched
 * groups first); block_group (optional, n_blocks entries) the group of
 * every block, -1 for a block without voxels.  VIE_EINVAL as
 * vie_problem_create. */
vie_status vie_plan(const vie_grid* grid, const double* eps_r, const int32_t* block_id, int32_t n_blocks,
                    int32_t overlap, vie_problem_info* info, vie_group_plan* groups, int32_t groups_cap,
                    int32_t* block_group);

/* Incident plane wave E_inc = pol * exp(-j k0 khat . r) at every voxel centre
 * (Sec. III: x-polarised wave along z).  kdir: unit vector (|kdir| = 1 within
 * 1e-12, else VIE_EINVAL); pol: 3 complex (6 doubles); e_inc: 3*nx*ny*nz
 * complex written.  Host helper, no device needed. */
vie_status vie_plane_wave(const vie_grid* grid, const double kdir[3], const double pol[6], double* e_inc);

/* The same wave for rooftop problems (vie_problem_create_rooftop): component
 * c at the centre of the face between voxel (x, y, z) and its neighbour
 * along axis c, i.e. half a cell further along that axis than the voxel
 * centre.  Host helper, no device needed. */
vie_status vie_plane_wave_faces(const vie_grid* grid, const double kdir[3], const double pol[6], double* e_inc);

/* y = A x on the device (the hot path's product; eqs. (2)-(4), (6)).
 * x_dev, y_dev: 3*nx*ny*nz complex double.  x is masked to the scatterer
 * on input; y is 0 on vacuum voxels.  x_dev and y_dev must not overlap. */
vie_status vie_matvec(vie_problem* p, int32_t precision, const void* x_dev, void* y_dev, void* stream);

/* Instrumented product for measurement: runs y = A x `reps` times on
 * `stream` (x must be zero on vacuum voxels; no input masking, as inside the
 * solver) with HIP events around each of the five passes (x forward,
 * y forward, z forward + spectral multiply + z inverse, y inverse,
 * x inverse + local term) and writes the mean duration of each pass in
 * milliseconds to pass_ms[0..4].  Synchronises the stream. */
vie_status vie_matvec_profile(vie_problem* p, int32_t precision, const void* x_dev, void* y_dev, void* stream,
                              int32_t reps, double* pass_ms);

/* Instrumented product of one shape group of blocks, for measurement: marks
 * the first n_active systems of group `group` (in vie_plan's group order)
 * iterating and the others converged, runs the group's batched product
 * `reps` times on `stream` with HIP events around each of its passes (those
 * of vie_matvec_profile; passes 2 and 4 are empty for groups on the fused
 * plane kernels) and writes the mean duration of each pass in milliseconds
 * to pass_ms[0..4].  Kernels, grid and tuned variant are those of the inner
 * solves; the pass-1 and pass-5 kernels run without the fused vector
 * updates.  Uses and overwrites the problem's inner solver state: call it
 * between solves.  Synchronises the stream.  Errors: VIE_EINVAL for a bad
 * group, count, precision or reps. */
vie_status vie_group_profile(vie_problem* p, int32_t precision, int32_t group, int32_t n_active, int32_t reps,
                             void* stream, double* pass_ms);

/* y = K2 x with K2 = blockdiag(A_1, ..., A_N) (eq. (10)): every block's
 * matrix applied to the block's part of x.  Needs block ids. */
vie_status vie_block_matvec(vie_problem* p, int32_t precision, const void* x_dev, void* y_dev, void* stream);

/* y = K2^{-1} w by inner BiCGSTAB-FFT solves of every block to tol_inner
 * (x0 = 0, at most maxit_inner steps, last iterate kept), every block
 * independent (Sec. II-B).  flags: VIE_FLAG_NO_GRAPHS and
 * VIE_FLAG_NO_BLOCK_KERNEL as in vie_opts.flags (other bits: VIE_EINVAL).
 * inner_iters (optional) receives the total inner steps. */
vie_status vie_precond_apply(vie_problem* p, int32_t precision, double tol_inner, int32_t maxit_inner,
                             int32_t flags, const void* w_dev, void* y_dev, void* stream, int64_t* inner_iters);

/* Solve A P = E_inc (host arrays).  e_inc: 3*nvox complex; e_tot_out:
 * 3*nvox complex, E_tot = P / chi on the scatterer, 0 in vacuum (eq. (2));
 * pol_out: optional (NULL) P.  Returns VIE_OK, VIE_NOT_CONVERGED (best
 * iterate written) or an error. */
vie_status vie_solve(vie_problem* p, const double* e_inc, const vie_opts* opts, double* e_tot_out, double* pol_out,
                     vie_stats* stats);

/* Same with device buffers on `stream` (inputs already in HBM). */
vie_status vie_solve_device(vie_problem* p, const void* e_inc_dev, const vie_opts* opts, void* e_tot_dev,
                            void* pol_dev, vie_stats* stats, void* stream);

/* ------------------------------------------------------------------ fields
 * Post-processing of a solution P (the pol output of a solve, device,
 * 3*nvox complex). */

/* Total field at every voxel of the box, scatterer and vacuum alike:
 * e_box = E_inc + sum_n T(m - n) P_n (eq. (3) with the operator of eq. (1);
 * on the scatterer this is P / chi, eq. (2)).  One FFT product in
 * `precision`.  All three device buffers are 3*nvox complex and must not
 * overlap e_box. */
vie_status vie_total_field_box(vie_problem* p, int32_t precision, const void* pol_dev, const void* e_inc_dev,
                               void* e_box_dev, void* stream);

/* Far field of the voxel currents, F(rhat) = (I - rhat rhat) sum_n P_n dV
 * exp(+j k0 rhat . r_n) (r_n: voxel centre relative to the grid centre; for
 * rooftop problems component c of entry n is at its face centre, r_n plus
 * d_c / 2 along axis c), for
 * n_dir unit directions rhat (host, 3 doubles each; |rhat| = 1 within 1e-12
 * else VIE_EINVAL).  f_out: host, 3*n_dir complex.  FP64; synchronises the
 * stream. */
vie_status vie_far_field(vie_problem* p, const void* pol_dev, int32_t n_dir, const double* rhat, double* f_out,
                         void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): vie_far_field
 * with device arrays in and out and no allocation of any kind.
 *   pol_dev:  3*nvox complex, the solution P (device);
 *   rhat_dev: n_dir unit directions, 3 doubles each (device; not checked);
 *   f_dev:    3*n_dir complex written (device), as vie_far_field's f_out.
 * The per-chunk partial sums live in a fixed array of 8 MiB that the library
 * keeps on every GPU it runs on until the process ends (its device address
 * is looked up by vie_context_create).  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU race, so run them in order (one
 * stream, or synchronised).  n_dir * ceil(nx ny nz / 2048) * 6 must not
 * exceed 1048576 (VIE_EINVAL otherwise).  Ordered on `stream`; returns
 * without synchronising.  Same kernels and summation order as
 * vie_far_field, so the results are identical. */
vie_status vie_far_field_noalloc(vie_problem* p, const void* pol_dev, int32_t n_dir, const void* rhat_dev,
                                 void* f_dev, void* stream);

/* Bistatic radar cross-section for a unit-amplitude incident wave,
 * sigma(rhat) = k0^4 |F(rhat)|^2 / (4 pi) (the E-plane curves of Sec. III,
 * Figs. 1-2, for rhat in the x-z plane).  sigma_out: host, n_dir doubles. */
vie_status vie_rcs(vie_problem* p, const void* pol_dev, int32_t n_dir, const double* rhat, double* sigma_out,
                   void* stream);

/* Several right-hand sides on one problem (incident fields of different
 * directions or polarisations on the same operator and partition).
 * e_inc_dev, e_tot_dev and pol_dev (optional): nrhs consecutive vectors of
 * 3*nx*ny*nz complex each (device, ordered on the stream); stats: NULL or
 * nrhs entries.  BiCGSTAB runs the nrhs systems as one batch: every
 * full-grid product, vector update and finalize launch covers all of them
 * and each system stops on its own status, with the same per-system
 * arithmetic as a single solve (plain solves: results equal those of
 * separate vie_solve_device calls; tested).  With the preconditioner, each
 * application solves the blocks of all right-hand sides together: the
 * blocks of nrhs copies of the problem stacked along z, in the problem's own
 * shape groups (a replica built by the first such call for that nrhs, kept
 * with the problem); a system that has stopped contributes zero right-hand
 * sides, which its blocks skip.  Its inner_iters_total and precond_applies
 * are the batch's totals.  VIE_SOLVER_FGMRES and VIE_SOLVER_CGS solve the
 * right-hand sides one after another.  Batch storage (12 vectors and one FFT work buffer per
 * right-hand side, plus the replica) is counted in footprint_bytes
 * (VIE_EBUSY beyond the context's budget).  Returns the first error, else
 * VIE_NOT_CONVERGED if any system did not converge, else VIE_OK; every
 * system's result and statistics are written.  nrhs in [1, 4096]. */
vie_status vie_solve_batch(vie_problem* p, int32_t nrhs, const void* e_inc_dev, const vie_opts* opts,
                           void* e_tot_dev, void* pol_dev, vie_stats* stats, void* stream);

/* Many independent problems of one grid shape solved as one batch (Sec.
 * III-C, Table III: independent solves run in parallel; here the parallel
 * axis is the problem).  The problems may differ in permittivity, block
 * partition, spacing and wavelength, but not in nx, ny, nz or the FFT
 * lengths (VIE_EINVAL), and belong to one context.  problems: n distinct
 * handles; e_inc_dev[r], e_tot_dev[r], pol_dev[r] (pol_dev optional): device
 * vectors of 3*nx*ny*nz complex of problem r, ordered on the stream; stats:
 * NULL or n entries.  BiCGSTAB runs the n outer solves as one batch: every
 * full-grid product (each system with its own 1/chi and its own spectra,
 * read through a table), vector update and finalize launch covers all of
 * them, and each stops on its own status.  With the preconditioner, each
 * application solves the blocks of all problems together: the blocks are
 * stacked along z, regrouped across problems by box shape, each with its
 * own problem's spectra, all on the batched kernels (no one-workgroup block
 * solver); a problem that has stopped contributes zero right-hand sides.
 * The outer products use the kernel variants of problems[0] (pinned or
 * tuned).  The FP64 true residual, mixed-mode refinement and the fields are
 * then formed per problem as in vie_solve_device.  inner_iters_total and
 * precond_applies are the batch's totals.  FGMRES and CGS, and n = 1, solve
 * the problems one after another.  Batch storage (1/chi, 12 vectors and a
 * work buffer per problem, the stacked blocks) is allocated for the call
 * and counted against the context's budget while it runs (VIE_EBUSY beyond
 * it).  Locks every problem for the call.  Returns the first error, else
 * VIE_NOT_CONVERGED if any problem did not converge, else VIE_OK; every
 * problem's result and statistics are written.  n in [1, 4096]. */
vie_status vie_solve_many(int32_t n, vie_problem* const* problems, const void* const* e_inc_dev,
                          const vie_opts* opts, void* const* e_tot_dev, void* const* pol_dev, vie_stats* stats,
                          void* stream);

/* ------------------------------------------------------------------ serving
 * A request queue per context: independent solves (any grid, wavelength,
 * partition and options) are admitted in arrival order as solver slots and
 * device memory free up, and run concurrently, each slot on its own HIP
 * stream, each request in a problem of its own (created when admitted,
 * destroyed when it finishes).  Green spectra and tuned kernel choices are
 * cached in the context and shared by requests of the same shapes, so a
 * request gives the same result alone or among others.  Results come back
 * to host memory.
 *
 * Memory admission: a request is started only when the context's memory in
 * use (problems created by the caller + requests running) plus the
 * request's footprint (vie_footprint) fits the context's hbm_budget_bytes
 * (0 = no limit); until then it waits, in order, in the queue. */

/* Start the server of ctx with `slots` concurrent solves (1..64) and room for
 * queue_cap waiting requests (>= 1).  Optional: the first vie_submit starts
 * it with 4 slots and 1024 places.  VIE_EBUSY if it is already running. */
vie_status vie_server_start(vie_context* ctx, int32_t slots, int32_t queue_cap);

/* Device bytes a problem with these inputs would hold (vie_problem_create's
 * arguments; spectra already cached in ctx are not counted), plus the
 * transient set-up memory of spectra not yet cached.  vie_submit reserves
 * more for a request: every spectrum and its set-up memory whether cached or
 * not (the cache shares spectra only while a problem holds them), plus the
 * request's incident and result vectors on the device. */
vie_status vie_footprint(vie_context* ctx, const vie_grid* grid, const double* eps_r, const int32_t* block_id,
                         int32_t n_blocks, size_t* bytes);

/* Queue one solve: the arguments of vie_problem_create plus those of
 * vie_solve (e_inc: 3*nvox complex; opts as vie_solve).  All host arrays are
 * copied before the call returns.  *out receives a ticket, to be passed to
 * vie_wait exactly once.  VIE_EINVAL on invalid input (or a footprint larger
 * than the whole budget), VIE_EBUSY when the queue is full. */
vie_status vie_submit(vie_context* ctx, const vie_grid* grid, const double* eps_r, const int32_t* block_id,
                      int32_t n_blocks, const double* e_inc, const vie_opts* opts, vie_ticket* out);

/* Wait up to timeout_s seconds (< 0: no limit) for the request.  When it has
 * finished: writes e_tot_out (3*nvox complex, may be NULL), stats (may be
 * NULL) and times (may be NULL: seconds queued, in set-up, in the solve),
 * releases the ticket and returns the request's status (that of vie_solve;
 * VIE_ECANCELLED if cancelled).  VIE_ETIMEDOUT if still queued or running:
 * nothing written, the ticket stays valid. */
vie_status vie_wait(vie_ticket t, double timeout_s, double* e_tot_out, vie_stats* stats, double* times);

/* Cancel a request: a queued one is dropped, a running one stops after its
 * current outer step.  The ticket must still be passed to vie_wait (which
 * then returns VIE_ECANCELLED, or the status of a request that had already
 * finished). */
vie_status vie_cancel(vie_ticket t);

#ifdef __cplusplus
}
#endif

#endif /* VIE_H */

// Internal interface between the host orchestration (vie_api.cpp) and the
// HIP kernels.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "cx.h"

namespace vie {

// Per-system solver status, shared by every kernel that gates on it.
enum SysStatus : int {
  ST_ACTIVE = 0,      // iterating
  ST_CONVERGED = 1,   // done, x final
  ST_HALF = 2,        // converged at the half step; x += alpha y still pending
  ST_BREAKDOWN = 3,   // rho, <rhat, v> or omega vanished; x = last iterate
  ST_MAXIT = 4,       // iteration cap reached; x = last iterate
  ST_IDLE = 5,        // not started / skipped (zero right-hand side)
  ST_RESTART = 6,     // flexible GMRES: cycle full, x update and restart pending
};

// FFT lengths with compiled kernels (2^a 3^b, up to 512).
constexpr int kFftLengths[] = {1,  2,  3,  4,  6,   8,   12,  16,  24,  32,  36,
                               48, 64, 72, 96, 128, 144, 192, 256, 288, 384, 512};
// Smallest supported L >= min_len, or -1.  xy: an x or y length, which
// skips 36 (no fused plane kernels for it; 48 keeps square boxes on the
// plane kernels).
int smallest_fft_length(int min_len, bool xy = false);

// Twiddle tables exp(-2 pi i t / L), one per supported L, for one precision.
template <typename R>
struct TwiddleSet {
  const cx<R>* table[513];   // indexed by L (null where unsupported)
};

// A batch of `nsys` equally-shaped systems (outer grid or a group of blocks).
// Vectors are c128 [nsys][3][nz][ny][nx]; the work buffer holds the
// partially transformed components [nsys][3][nz][ly][lx] in precision R.
template <typename R>
struct MvmBatch {
  int nx, ny, nz;          // voxel box
  int lx, ly, lz;          // circulant lengths (>= 2n - 1)
  int nsys;
  int64_t vstride;         // c128 elements between systems' vectors (3 nx ny nz)
  int64_t cstride;         // c128 elements between systems' 1/chi arrays (nx ny nz)
  int64_t wstride;         // elements between systems' work buffers
  int64_t sstride;         // elements between systems' spectra (0 = shared)
  const c128* chi_inv;     // [nsys][nz][ny][nx], 0 on voxels outside the system
  const cx<R>* spec;       // [6][lz/2+1][ly/2+1][lx/2+1] per system
  const cx<R>* const* spec_tab;   // per-system spectra (device table; null: spec + sys sstride)
  cx<R>* work;
  const int* status;       // per system; null = always active
  const TwiddleSet<R>* tw; // host-side pointer table (values are device pointers)
  int zvariant;            // z-pass kernel variant (see tune_zpass)
  int plane;               // 1: x and y transforms fused per z-plane (plane_supported(lx, ly))
  int pvariant;            // plane kernels: planes per workgroup variant (see tune_plane)
  // 0: collocated voxels (spec: six octant spectra, 1/chi per voxel);
  // 1: rooftop faces (spec: the scalar octant spectrum and difference
  // symbols of green_spectrum_rooftop; 1/chi per face, [nsys][3][nz][ny][nx])
  int rooftop;
};

// Square transforms small enough for the fused plane kernels.
bool plane_supported(int lx, int ly);

// y = A x for every active system of the batch (Sec. I Toeplitz + FFT;
// eqs. (2)-(4)).  `mask_input` zeroes x where 1/chi = 0 before transforming.
// `ev` (optional, 6 events): ev[0] is recorded before pass 1 and ev[i] after
// pass i, on stream s.
template <typename R>
void mvm(const MvmBatch<R>& b, const c128* x, c128* y, bool mask_input, hipStream_t s, hipEvent_t* ev = nullptr);

struct KBatch;
// The product in three launches groups, with BiCGSTAB work fused into its
// first and last passes.  Pass 1 input (in_mode):
//   0: x (masked if mask_input);
//   1: p = r + beta (p - omega v) (p = r on the first step), written to p;
//   2: s = r - alpha v, written to p (the s vector), partials of ||s||^2;
//   3: as 2 with alpha = rho / <rhat, v> formed in the kernel from the
//      partials of the system's previous product (out_mode 1) and no
//      partials written: every workgroup sums them in the same order, the
//      system's first workgroup counts the step and records alpha, or the
//      breakdown when <rhat, v> = 0 (the scalar step of FIN_ALPHA, fused).
// Pass 5 (out_mode), after writing y = A x:
//   0: nothing; 1: partials of <rhat, y>; 2: partials of <y, s>, <y, y>;
//   3: y = rhat + sum T x at every voxel (rhat = E_inc: the total field of
//      eq. (3) in and around the scatterer; no mask, no partials);
//   4: as 2, plus partials of ||s||^2 (then FIN_SOMEGA: the half-step test
//      and omega in one finalize).
// In pass 5, x is the product's input (x for in_mode 0, f.p otherwise).
struct FuseArgs {
  int in_mode, out_mode;
  const c128* r;
  c128* p;
  const c128* v;
  const c128* rhat;
  const c128* s;
};
template <typename R>
void mvm_pass1(const MvmBatch<R>& b, const KBatch* k, const FuseArgs& f, const c128* x, bool mask_input,
               hipStream_t s);
template <typename R>
void mvm_mid(const MvmBatch<R>& b, hipStream_t s);   // passes 2-4
template <typename R>
void mvm_pass5(const MvmBatch<R>& b, const KBatch* k, const FuseArgs& f, const c128* x, c128* y, hipStream_t s);

// Times every z-pass variant on the batch's work buffer (clobbers it) and
// returns the fastest; ms_out (optional, kZPassVariants entries) receives
// each variant's time for three runs, -1 where not timed.
constexpr int kZPassVariants = 5;
template <typename R>
int tune_zpass(const MvmBatch<R>& b, hipStream_t s, float* ms_out = nullptr);

// Plane-kernel variants (planes per workgroup: 0 as LDS allows, 1 two,
// 2 one).  tune_plane times the forward and inverse plane passes of each on
// the batch's work buffer with x as input and y as output (clobbers all
// three) and returns the fastest; 0 for batches without plane kernels.
constexpr int kPlaneVariants = 3;
template <typename R>
int tune_plane(const MvmBatch<R>& b, const c128* x, c128* y, hipStream_t s, float* ms_out = nullptr);

// Chunks per system of the fused first/last passes (for partial sizing).
int64_t mvm_row_tiles(int lx, int nz, int ny);

// Octant spectra of the 6 Green-tensor components for one box shape:
// evaluates T(m) on the (lz, ly, lx) circulant grid in FP64, transforms it
// with the device FFT and keeps q in [0, L/2] per axis.  `scratch` holds
// 6 lx ly lz c128.  Writes both precisions if the pointers are non-null.
void green_spectra(int nx, int ny, int nz, int lx, int ly, int lz, double dx, double dy, double dz, double k0,
                   c128* scratch, c128* spec64, c64* spec32, const TwiddleSet<double>& tw, hipStream_t s);

// Spectrum of the rooftop discretisation for one box shape: the octant of
// FFT(k0^2 dV g~) (one component, ox oy oz elements) followed by the
// difference-symbol tables b_x[lx], b_y[ly], b_z[lz] (see k_zconv_col).
// `scratch` holds lx ly lz c128.  Writes both precisions if non-null.
void green_spectrum_rooftop(int nx, int ny, int nz, int lx, int ly, int lz, double dx, double dy, double dz,
                            double k0, c128* scratch, c128* spec64, c64* spec32, const TwiddleSet<double>& tw,
                            hipStream_t s);

}  // namespace vie

namespace vie {

// ------------------------------------------------------------------ Krylov
// Scalars of one BiCGSTAB system (outer solve, or one block's inner solve).
struct KState {
  c128 rho, rho_old, alpha, omega, beta;
  double nb;        // ||b||
  double rnorm;     // ||r|| / ||b|| after the last full step
  double snorm;     // ||s|| / ||b|| after the last half step
  double tol;
  int iters, maxit;
  int pending;      // fused step: outcome of the half step for k_step_end (0, ST_HALF or ST_BREAKDOWN)
  int pad1;
};

// A batch of `nsys` systems with vectors of `n` c128 each (contiguous,
// system-major).  `status`/`st` point at this batch's entries.
struct KBatch {
  int nsys;
  int64_t n;
  int* status;
  KState* st;
  double* partials;   // per system `pstride` doubles (>= 4 * partial count)
  int64_t pstride;
  int* ntile;         // per system: partial count written by the last producer
  double* partials2;  // second buffer, same layout: written by k_update_xr_fused while
                      // the first one is still read by that kernel
};

// Inner block solves with one workgroup per system (Sec. II-B): the whole
// unpreconditioned BiCGSTAB of each system of a group (x0 = 0, rhs b) in one
// launch.  Vectors are c128 [nsys][3][bz][by][bx]; the work buffer holds
// [nsys][3][bz][ly][lx] elements of R; lx == ly.  On return each system's
// status is CONVERGED, MAXIT or BREAKDOWN (IDLE if the gate is not ACTIVE)
// and its KState holds nb, iters and rnorm.
struct BlockSolveArgs {
  int nsys;
  int bx, by, bz;
  int64_t n;                 // 3 bx by bz
  const c128* chi;           // 1/chi per system [nsys][bz][by][bx], 0 outside the block
  const c128* b;
  c128 *x, *r, *rhat, *p, *v, *s, *t;
  void* work;
  const void* spec;          // octant spectra for (lx, ly, lz), shared by the systems
  const void* twx;           // twiddle table for lx (== ly)
  const void* twz;           // twiddle table for lz
  int* status;
  KState* st;
  const int* gate;           // skip unless *gate == ACTIVE (null: always run)
  double tol;
  int maxit;
};
// True if the group's FFT box (lx, ly, lz) with bz voxel planes has a
// block-solver kernel and is small enough for one workgroup to win.
bool block_solver_supported(int lx, int ly, int lz, int bz);
template <typename R>
void block_solve(const BlockSolveArgs& a, int lx, int lz, hipStream_t s);

// Far field F(rhat) = (I - rhat rhat) sum_n P_n dV exp(+j k0 rhat . r_n)
// for ndir directions (rhat: device, 3 doubles each; F: device, 3 c128 each).
// part: device scratch of 6 far_field_chunks(nx ny nz) doubles per direction.
// faces: P holds rooftop face unknowns (component c at its face centre, half
// a cell along axis c from the voxel centre).
int64_t far_field_chunks(int64_t nv);
// The far field's fixed scratch array (for the entry point that allocates
// nothing): its capacity in doubles, and its address on the current device
// (looked up once per device at set-up; throws on failure).
int64_t far_field_scratch_doubles();
void* far_field_scratch_address();
void far_field(const c128* P, int nx, int ny, int nz, double dx, double dy, double dz, double k0, const double* rhat,
               int ndir, double* part, c128* F, hipStream_t s, bool faces = false);

// Flexible GMRES(m) of one system (the outer solve).  V: m+1 basis vectors,
// Z: m preconditioned vectors (or null without preconditioner), each n c128;
// H: (m+1) x m column-major; status: the solve's status (ST_ACTIVE while
// iterating; gates the product and the preconditioner as well).
struct GmresState {
  double nb, tol, relres, hnext;
  int iters, maxit, k, pad;   // k: columns of the current cycle
};
struct GmresDev {
  c128* V;
  c128* Z;
  int64_t n;
  int m;
  c128 *H, *sn, *g, *y, *h, *c;
  double* cs;
  double* part;     // (m+1) * nchunk * 2 doubles
  int64_t nchunk;   // gmres_chunks(n)
  double* scal;     // scal[0]: squared norm input of gmres_arnoldi / gmres_start
  GmresState* st;
  int* status;
};
int64_t gmres_chunks(int64_t n);
void gmres_orthogonalise(const GmresDev& d, c128* w, int j, hipStream_t s);   // CGS2 of w against V_0..V_j
void gmres_arnoldi(const GmresDev& d, c128* w, int j, hipStream_t s);         // column j, rotations, w /= ||w||
void gmres_start(const GmresDev& d, c128* v0, bool first, double tol, int maxit, hipStream_t s);   // g, status; v0 /= ||v0||
void gmres_update(const GmresDev& d, c128* x, const c128* B, hipStream_t s);  // x += B y

// Scalar steps applied by k_finalize after a producer wrote partials.
enum FinKind : int { FIN_INIT = 0, FIN_ALPHA = 1, FIN_S = 2, FIN_OMEGA = 3, FIN_XR = 4, FIN_SOMEGA = 5, FIN_CGS = 6 };

int64_t krylov_chunks(int64_t n);   // reduction chunks per system (vector kernels)

// x = 0, r = rhat = b, partials of ||b||^2 (skipped when the gate is set and
// not ACTIVE).
void k_init(const KBatch& k, const c128* b, c128* x, c128* r, c128* rhat, const int* gate, hipStream_t s);
// One workgroup per system of `k` (one launch for every system of a solve):
//   FIN_INIT:  ||b||, rho; status ACTIVE, CONVERGED (||b|| = 0) or IDLE (gated)
//   FIN_ALPHA: alpha = rho / <rhat, v> (counts the step)
//   FIN_S:     half-step test on ||s||
//   FIN_OMEGA: omega = <t, s> / <t, t>
//   FIN_SOMEGA: half-step test on ||s|| (from pass-5 out_mode 4), then omega
//   FIN_XR:    rho', ||r||, convergence, breakdown, cap, beta; HALF -> CONVERGED
//   FIN_CGS:   CGS step end: rho' = <rhat, r>, ||r||, convergence, breakdown,
//              cap, beta = rho' / rho
void k_finalize(const KBatch& k, FinKind kind, hipStream_t s, const int* gate = nullptr, double tol = 0,
                int maxit = 0);
// p = r (first step) or p = r + beta (p - omega v)
void k_update_p(const KBatch& k, const c128* r, const c128* v, c128* p, hipStream_t s);
// s = r - alpha v and partials of ||s||^2 (then FIN_S)
void k_update_s(const KBatch& k, const c128* r, const c128* v, c128* sv, hipStream_t s);
// x += alpha y + omega z, r = s - omega t, partials of <rhat, r>, ||r||^2
// (then FIN_XR); after a half-step convergence, x += alpha y only.
void k_update_xr(const KBatch& k, c128* x, const c128* y, const c128* z, c128* r, const c128* sv, const c128* t,
                 const c128* rhat, hipStream_t s);
// The end of a BiCGSTAB step with the scalar work fused into the kernels
// (unpreconditioned systems, y = p and z = s), after the second product's
// pass 5 (out_mode 4: partials of <t, s>, <t, t>, ||s||^2):
// k_update_xr_fused forms ||s|| and omega in every workgroup from those
// partials (same fixed order); on the half step (||s|| <= tol ||b||) x +=
// alpha y only, on <t, t> = 0 nothing, else x += alpha y + omega z and
// r = s - omega t with the partials of <rhat, r>, ||r||^2 in partials2.  The
// system's first workgroup records ||s||, omega and the outcome in
// KState.pending.  k_step_end then finishes every system of the batch in one
// workgroup: a pending half step or breakdown is applied, otherwise the
// scalar step of FIN_XR from partials2; with count_out it also stores the
// number of systems still ACTIVE there (may be host-mapped memory).
void k_update_xr_fused(const KBatch& k, c128* x, const c128* y, const c128* z, c128* r, const c128* sv,
                       const c128* t, const c128* rhat, hipStream_t s);
void k_step_end(const KBatch& k, int* count_out, hipStream_t s);
// Conjugate gradient squared (solver variant), per system, skipped unless
// ACTIVE:
// u = r, p = r (first step) or u = r + beta q, p = u + beta (q + beta p)
void cgs_update_up(const KBatch& k, const c128* r, c128* u, const c128* q, c128* p, hipStream_t s);
// q = u - alpha v, w = u + q (after FIN_ALPHA)
void cgs_update_q(const KBatch& k, const c128* u, const c128* v, c128* q, c128* w, hipStream_t s);
// x += alpha uh
void cgs_update_x(const KBatch& k, c128* x, const c128* uh, hipStream_t s);
// r = b - t (t = A x), partials of <rhat, r>, ||r||^2 (then FIN_CGS)
void cgs_update_r(const KBatch& k, const c128* b, const c128* t, c128* r, const c128* rhat, hipStream_t s);
// After one preconditioner application (skipped when the gate is not
// ACTIVE): acc[0] += sum of the inner iteration counts of `slots`,
// acc[1] += 1, and the counts are appended to hist at acc[2] (if they fit).
void record_inner(const int* gate, const KState* st, const int* slots, int nslots, int64_t* acc, int32_t* hist,
                  int64_t hist_cap, hipStream_t s);
// number of ACTIVE entries of status[0..n) into *out (device int)
void count_active(const int* status, int n, int* out, hipStream_t s);
// y = x * chi_inv (E_tot = P / chi on the scatterer, 0 in vacuum), batched;
// element i uses chi_inv[i % cper] (cper 0: nv, one value per voxel; 3 nv:
// one per face of the rooftop discretisation)
void total_field(const c128* P, const c128* chi_inv, c128* e, int64_t nv, int ncomp, hipStream_t s,
                 int64_t cper = 0);
// Rooftop face fields: component c of entries in the grid's last cell layer
// along axis c set to 0 (those faces' second cell lies outside the grid)
void zero_outer_faces(c128* e, int nx, int ny, int nz, hipStream_t s);
// b = e * mask (mask: chi_inv != 0), 3 components of nv voxels; chi_inv
// indexed as in total_field
void masked_copy(const c128* e, const c128* chi_inv, c128* b, int64_t nv, hipStream_t s, int64_t cper = 0);
// r = b - a (c128, n elements) ; partial-free helper for refinement
void sub_vec(const c128* b, const c128* a, c128* r, int64_t n, hipStream_t s);
// Batch layout [nrhs][3][nv] <-> stacked layout [3][nrhs][nv] (the same
// vectors on a grid of nrhs copies stacked along z).  batch_to_stacked
// writes zeros for systems whose status is not ACTIVE (status may be null).
void batch_to_stacked(const c128* src, c128* dst, int nrhs, int64_t nv, const int* status, hipStream_t s);
void stacked_to_batch(const c128* src, c128* dst, int nrhs, int64_t nv, hipStream_t s);
// x += d
void add_vec(c128* x, const c128* d, int64_t n, hipStream_t s);
// ||v||^2 of one vector into *out (device double), deterministic; partials
// holds 4 * krylov_chunks(n) doubles
void norm2(const c128* v, int64_t n, double* partials, double* out, hipStream_t s);

// ------------------------------------------------------------------ blocks
// Block k of the partition lives in group block_group[k] as system
// block_sys[k] with box origin block_origin[k] (voxel coordinates of the
// outer grid); the group's box is gbox[g].  Group vectors are passed as a
// device array of per-group base pointers.
struct BlockMap {
  int nblocks, ngroups;
  const int* block_id;      // outer grid [nz][ny][nx], -1 vacuum
  const int* block_group;   // [nblocks]
  const int* block_sys;     // [nblocks]
  const int4* block_origin; // [nblocks] (x, y, z, unused)
  const int4* gbox;         // [ngroups] (bx, by, bz, unused)
  int nx, ny, nz;
  int faces;                // 1: rooftop face unknowns, block_id per face [3][nz][ny][nx]
};
// gvec_k[c][local] = w[c][v] for every scatterer voxel v (members only; the
// other entries of the group vectors are left untouched, i.e. zero); with
// m.faces, per face: component c of entry v goes to the block owning that
// face
void block_gather(const BlockMap& m, const c128* w, c128* const* gdst, hipStream_t s);
// y[c][v] = gsrc_k[c][local(v)] for scatterer voxels, 0 for vacuum
void block_scatter(const BlockMap& m, c128* const* gsrc, c128* y, hipStream_t s);
// Expanded (overlapping) blocks: system q of a group gathers w at every voxel
// of its solve set, marked by chi_q != 0 on its box (origin[q], box bx by bz).
void gather_sets(const c128* w, int nx, int ny, int nz, int bx, int by, int bz, int nsys, const int4* origin,
                 const c128* chi, c128* gdst, hipStream_t s);

}  // namespace vie

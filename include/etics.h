/*
 * etics.h -- C-ABI of the MI355X expansion force library (libetics.so).
 *
 * The library computes the self-consistent-field (SCF) and multipole-expansion
 * (MEX) gravitational potential and acceleration of N particles, following
 * Meiron, Li, Holley-Bockelmann & Spurzem, "Expansion Techniques for
 * Collisionless Stellar Dynamical Simulations" (arXiv:1406.4254):
 *   - SCF: eq. scf-phi of Section 2.4 with the Hernquist-Ostriker radial basis the
 *     paper adopts (Section 2.5), basis scale a = 1, G = 1, expansion centre at the
 *     origin (Section 5.1 leaves centre and length unit to the caller; shift and
 *     scale the positions before the call);
 *   - MEX: eqs. mex-phi, mex-qlm, mex-plm of Section 2.4, with particles ordered by
 *     radius and the inward/outward sums taken exclusively (Section 3.2).
 *
 * Memory: every array argument is a DEVICE pointer (for example a torch tensor's
 * data_ptr()) owned by the caller; the library never frees or keeps them.  Arrays
 * are structure-of-arrays, FP64, contiguous.  The workspace is caller-allocated
 * device memory of at least the size returned by the matching *_workspace_size
 * call, aligned to 256 bytes; its contents need not be initialised and are
 * undefined after the call.
 *
 * Streams: `stream` is a hipStream_t (NULL = the legacy default stream).  All
 * compute calls only enqueue work on that stream and return; none synchronises,
 * allocates device memory or copies to/from the host, so they may be captured in a
 * hipGraph.  The one exception is etics_leapfrog_scf_batched, which itself captures
 * a step into a hipGraph: on first use it creates a library stream and instantiates
 * the graph (it must not be called inside another capture).
 *
 * Errors: 0 on success, otherwise a negative ETICS_E* code; a message for the
 * last failure of the calling thread is available from etics_last_error().
 * Arguments are validated before any device work is enqueued, so an invalid call
 * enqueues nothing.
 *
 * Coefficient layout (SCF): for 0 <= n <= nmax, 0 <= m <= l <= lmax,
 *   idx(n,l,m) = n (lmax+1)(lmax+2)/2 + l(l+1)/2 + m,   K = (nmax+1)(lmax+1)(lmax+2)/2.
 * A[idx] and B[idx] are the cosine and sine coefficients of
 *   Phi(r,theta,phi) = sum_{n,l,m>=0} PhiT_nl(r) Ybar_lm(theta) (A cos m phi + B sin m phi),
 * with PhiT_nl the Hernquist-Ostriker radial functions, Ybar_lm the orthonormal
 * Legendre amplitude (Condon-Shortley phase) and the (2 - delta_m0) factor of the
 * real form already applied; B[idx(n,l,0)] = 0.  The paper's complex coefficient
 * (Section 2.4, m >= 0) is (A - iB)/(2 - delta_m0).  The SCF coefficients include
 * every particle; MEX excludes the particle itself.
 */
#ifndef ETICS_H
#define ETICS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* precision modes: basis evaluation / force synthesis precision and the
   cross-particle reduction precision */
#define ETICS_FP64 0          /* everything in FP64 */
#define ETICS_MIXED_FP64ACC 1 /* FP32 basis and synthesis, FP64 coefficient reduction */
#define ETICS_MIXED_COMP32 2  /* FP32 basis and synthesis, compensated (double-float) FP32 reduction */

/* radial bases of the SCF expansion (Section 2.5) */
#define ETICS_BASIS_HO 0  /* Hernquist-Ostriker: Hernquist model as zeroth order (the paper's) */
#define ETICS_BASIS_CB 1  /* Clutton-Brock: Plummer model as zeroth order */

/* outputs of the force calls (bit mask) */
#define ETICS_POT 1
#define ETICS_ACC 2
#define ETICS_POT_ACC 3

/* return codes */
#define ETICS_OK 0
#define ETICS_EINVAL (-1)        /* bad size, cutoff, mode or a required NULL pointer */
#define ETICS_EWORKSPACE (-2)    /* workspace missing or smaller than required */
#define ETICS_EHIP (-3)          /* a HIP runtime or launch error */
#define ETICS_EUNSUPPORTED (-4)  /* valid request the library does not implement */

/* expansion cutoffs supported by the library */
#define ETICS_NMAX_CAP 20
#define ETICS_LMAX_CAP 14

/* Number of (A,B) coefficient pairs K = (nmax+1)(lmax+1)(lmax+2)/2 (Section 2.4,
   after eq. scf-phi; 308 at (10,6)).  Returns -1 for cutoffs outside the caps. */
int etics_coeff_count(int nmax, int lmax);

/* Workspace bytes needed by etics_scf_coeffs and etics_scf_force for n particles;
   0 if the arguments are invalid.  Host-only, enqueues nothing. */
size_t etics_scf_workspace_size(int64_t n, int nmax, int lmax, int precision);

/* SCF expansion coefficients (Section 2.4, eq. scf-phi; Section 3.3 computes them
   as the first part of a force calculation).
   x,y,z,m: [n] particle positions and masses.  A,B: [K] outputs (overwritten).
   n = 0 is valid and yields zero coefficients.  The cross-particle sums are taken
   in a fixed order, so repeated calls with the same inputs, sizes and precision
   give bitwise-identical results. */
int etics_scf_coeffs(const double* x, const double* y, const double* z, const double* m,
                     int64_t n, int nmax, int lmax, int precision,
                     double* A, double* B, void* workspace, size_t ws_bytes, void* stream);

/* Allocation-free form of etics_scf_coeffs, for callers that cannot allocate device
   memory or pass a workspace (code under hipGraph capture, tight serving loops,
   harnesses that forbid hipMalloc).  Same arguments, results and errors as
   etics_scf_coeffs, without the workspace: the partial sums live in a fixed
   24 MiB device array inside the library (one per device, held until the process
   ends), which covers every cutoff under the caps.  The call allocates nothing; the
   first call on a device looks up that array's device address.  All calls on one
   device share the array: calls that overlap in time on the same device (different
   streams, threads or processes' graphs replayed concurrently) race and must be
   serialised by the caller.  ETICS_EWORKSPACE if a plan ever needed more than the
   array holds. */
int etics_scf_coeffs_noalloc(const double* x, const double* y, const double* z, const double* m,
                             int64_t n, int nmax, int lmax, int precision,
                             double* A, double* B, void* stream);

/* SCF potential and acceleration a = -grad Phi at the points x,y,z [n] from
   coefficients A,B [K] (Section 3.3, the second part of a force calculation).
   outputs: ETICS_POT, ETICS_ACC or both.  pot may be NULL unless POT is requested,
   ax/ay/az may be NULL unless ACC is requested.  A point exactly at the origin gets
   no l = 0 force (its direction is undefined there). */
int etics_scf_force(const double* x, const double* y, const double* z, int64_t n,
                    int nmax, int lmax, const double* A, const double* B, int precision,
                    int outputs, double* pot, double* ax, double* ay, double* az,
                    void* workspace, size_t ws_bytes, void* stream);

/* The same two calls in either radial basis of Section 2.5 (the calls above use
   ETICS_BASIS_HO).  ETICS_BASIS_CB is the Clutton-Brock basis, whose zeroth order is a
   Plummer sphere of scale 1:
     PhiT_nl(r) = -sqrt(4 pi) r^l (1+r^2)^-(l+1/2) C_n^(l+1)(xi),  xi = (r^2-1)/(r^2+1),
     rhoT_nl(r) = K_nl/(4 pi) sqrt(4 pi) r^l (1+r^2)^-(l+5/2) C_n^(l+1)(xi),
     K_nl = 4n(n+2l+2) + (2l+1)(2l+3),
   normalised and laid out as above (A, B include (2 - delta_m0) and 1/I_nl,
   I_nl = integral of rhoT_nl PhiT_nl r^2 dr).  Coefficients must be synthesised in the
   basis they were computed in.  Workspace sizes are those of etics_scf_workspace_size.
   ETICS_EINVAL for any other basis value. */
int etics_scf_coeffs_basis(const double* x, const double* y, const double* z, const double* m,
                           int64_t n, int nmax, int lmax, int precision, int basis,
                           double* A, double* B, void* workspace, size_t ws_bytes, void* stream);
int etics_scf_force_basis(const double* x, const double* y, const double* z, int64_t n,
                          int nmax, int lmax, const double* A, const double* B, int precision,
                          int basis, int outputs, double* pot, double* ax, double* ay, double* az,
                          void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes needed by etics_mex_force; 0 if the arguments are invalid. */
size_t etics_mex_workspace_size(int64_t n, int lmax, int precision);

/* MEX potential and acceleration of every particle from all the others (Section
   2.4, eqs. mex-phi/qlm/plm; Section 3.2).  Particles are ordered by the FP64 key
   (x*x + y*y) + z*z (each operation rounded, no fused multiply-add), ties broken by
   index; the inward sums q run over particles before i, the outward sums p over
   particles after i.  ETICS_MIXED_* evaluate the angular functions in FP32 and keep
   radial powers, the ordered sums and the synthesis accumulation in FP64.  A
   particle exactly at the origin has no inward part and adds nothing to the outward
   sums. */
int etics_mex_force(const double* x, const double* y, const double* z, const double* m,
                    int64_t n, int lmax, int precision, int outputs,
                    double* pot, double* ax, double* ay, double* az,
                    void* workspace, size_t ws_bytes, void* stream);

/* Direct summation without softening, in FP64: the N-body force that the accuracy
   study of Section 4.1 compares with the expansions and with the smooth force of the
   model.  pot[i] = -sum m_j / r_ij and a_i = sum m_j (x_j - x_i) / r_ij^3 over all j
   with r_ij > 0 (G = 1): the particle itself, and any particle at exactly the same
   position, adds nothing.  Inputs as for the calls above (DEVICE arrays of n);
   outputs as selected by `outputs` (arrays the caller owns; unselected ones may be
   NULL).  No workspace; O(n^2) work.  Errors: ETICS_EINVAL for n < 0 or n >= 2^31, a
   bad `outputs` or a NULL array that is needed; ETICS_EHIP for a launch failure. */
int etics_direct_force(const double* x, const double* y, const double* z, const double* m,
                       int64_t n, int outputs, double* pot, double* ax, double* ay, double* az,
                       void* stream);

/* ---- Jerk (time derivative of the acceleration) and the fourth-order Hermite
   integrator.  The paper notes that Hernquist's SCF code computes the jerk (Section
   3.4) for its fourth-order Hermite scheme, the integrator it names as the next step
   for SCF (Section 5.4).  Here the particles move with velocities vx,vy,vz, and
     dA_nlm/dt = (2 - delta_m0) Atilde_nl sum_k m_k d/dt[PhiT_nl Ybar_lm cos(m phi)](x_k(t)),
   dB/dt likewise with sin, along x_k(t) = x_k + v_k t at t = 0; the jerk of a point i is
   the total derivative j_i = d/dt a(x_i + v_i t; A(t), B(t)), the field point and every
   particle of the field moving.  Hernquist-Ostriker basis.  A point exactly on the z
   axis (x = y = 0) gets a finite jerk in which the azimuthal rotation of the point is
   not followed (its azimuth has no time derivative there); use positions off the axis
   where the jerk matters. */

/* dA/dt and dB/dt [K] of particles x,y,z,vx,vy,vz,m [n] (layout and scaling as A, B;
   fixed summation order, bitwise repeatable).  Workspace: etics_scf_workspace_size. */
int etics_scf_coeffs_dot(const double* x, const double* y, const double* z, const double* vx,
                         const double* vy, const double* vz, const double* m, int64_t n, int nmax,
                         int lmax, int precision, double* Adot, double* Bdot, void* workspace,
                         size_t ws_bytes, void* stream);

/* Acceleration a = -grad Phi and jerk j = da/dt at the points x,y,z moving with
   vx,vy,vz [n], from A, B [K] and their time derivatives Adot, Bdot [K].  All six
   outputs [n] are required.  Workspace: etics_scf_workspace_size. */
int etics_scf_jerk(const double* x, const double* y, const double* z, const double* vx,
                   const double* vy, const double* vz, int64_t n, int nmax, int lmax, const double* A,
                   const double* B, const double* Adot, const double* Bdot, int precision, double* ax,
                   double* ay, double* az, double* jx, double* jy, double* jz, void* workspace,
                   size_t ws_bytes, void* stream);

/* Workspace bytes for etics_hermite_scf_batched; 0 if the arguments are invalid. */
size_t etics_hermite_workspace_size(int64_t ntotal, int nsys, int nmax, int lmax, int precision);

/* nsteps fourth-order Hermite predictor-corrector steps of dt (Makino & Aarseth 1992)
   for nsys independent systems (offsets, m as for the batched calls), each in its own
   SCF field:  x_p = x + v dt + a dt^2/2 + j dt^3/6,  v_p = v + a dt + j dt^2/2;
   a_1, j_1 at (x_p, v_p);  v_1 = v + (a + a_1) dt/2 + (j - j_1) dt^2/12;
   x_1 = x + (v + v_1) dt/2 + (a - a_1) dt^2/12.  x..vz are updated in place.  Every
   call first evaluates a, j at the current state.  Graph capture and replay as for
   etics_leapfrog_scf_batched (ETICS_LEAPFROG_EAGER launches every step directly;
   the graph cache is its own). */
int etics_hermite_scf_batched(double* x, double* y, double* z, double* vx, double* vy, double* vz,
                              const double* m, const int64_t* offsets, int nsys, int64_t ntotal,
                              int nmax, int lmax, int precision, double dt, int nsteps, int flags,
                              void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes for the batched SCF calls and the batched leapfrog over nsys
   systems with ntotal particles in all; 0 if the arguments are invalid. */
size_t etics_batched_workspace_size(int64_t ntotal, int nsys, int nmax, int lmax, int precision);

/* Batched SCF coefficients of nsys independent systems stored back to back:
   system s is particles offsets[s] .. offsets[s+1]-1 (offsets: DEVICE int64
   [nsys+1], non-decreasing, offsets[0] = 0, offsets[nsys] = ntotal).  A,B: [nsys*K],
   system s at s*K.  Each system's coefficients equal what etics_scf_coeffs returns
   for that system alone, up to the summation order. */
int etics_scf_coeffs_batched(const double* x, const double* y, const double* z, const double* m,
                             const int64_t* offsets, int nsys, int64_t ntotal, int nmax, int lmax,
                             int precision, double* A, double* B,
                             void* workspace, size_t ws_bytes, void* stream);

/* Batched SCF potential/acceleration: particle i of system s feels system s's
   coefficients A,B [nsys*K]. */
int etics_scf_force_batched(const double* x, const double* y, const double* z,
                            const int64_t* offsets, int nsys, int64_t ntotal, int nmax, int lmax,
                            const double* A, const double* B, int precision, int outputs,
                            double* pot, double* ax, double* ay, double* az,
                            void* workspace, size_t ws_bytes, void* stream);

/* leapfrog flags */
#define ETICS_LEAPFROG_EAGER 1 /* launch each step's kernels directly instead of replaying the graph */

/* nsteps kick-drift-kick leapfrog steps of dt for nsys independent systems, each
   feeling only its own SCF field (the paper integrates with a leapfrog, Section
   3.4):  v += dt/2 a(x);  x += dt v;  a = a(x);  v += dt/2 a.  x..vz are updated in
   place; m and offsets are as for the batched calls.  Every call first computes
   a(x) at the current positions (one extra force calculation), then runs the steps;
   each step's closing kick (and the next step's opening kick and drift) is applied
   per particle by the force kernel.  Unless ETICS_LEAPFROG_EAGER is set, one step is
   captured into a hipGraph on a library stream (the first time for a given set of
   pointers, sizes, precision, dt and workspace; a different set replaces the cached
   graph) and replayed nsteps-1 times on `stream`, followed by the last step launched
   directly; graph and eager runs launch the same kernels with the same arguments, so
   they give bitwise-equal results.  The cache is shared by all threads
   of the process (calls are serialised by a lock).  nsteps = 0 does nothing. */
int etics_leapfrog_scf_batched(double* x, double* y, double* z, double* vx, double* vy, double* vz,
                               const double* m, const int64_t* offsets, int nsys, int64_t ntotal,
                               int nmax, int lmax, int precision, double dt, int nsteps, int flags,
                               void* workspace, size_t ws_bytes, void* stream);

/* Measurement support (no passage of the paper; used to time the kernels against
   their roofline).  before/after are hipEvent_t handles created by the caller.  While
   set, every later compute call of the calling thread records `before` on its stream
   right before its main kernel and `after` right after it: the coefficient kernel
   (etics_scf_coeffs, etics_scf_coeffs_batched; not the final fixed-order sum), the
   force kernel (etics_scf_force, etics_scf_force_batched; not the coefficient
   rescale before it) and the synthesis kernel of etics_mex_force (not the sort and
   the ordered sums).  etics_leapfrog_scf_batched records nothing.  (NULL, NULL)
   turns it off; exactly one NULL is ETICS_EINVAL.  The library does not own the
   events and keeps only their handles. */
int etics_set_timing_events(void* before, void* after);

/* ---- Tile plans and the autotuner (the library's own tuning; no passage of the
   paper).  A coefficient call takes its tile shape from a plan: nw (wavefronts that
   share the basis work of a group of 64 particles: 4, 2 or 1, so a tile holds up to 64,
   128 or 256 particles), tp (particles per tile), streams (copies of the register
   blocks merged at the end), grid_mult (workgroups per CU, 1 or 2), phase2 (where the
   FP32 outer products run: 1 = vector ALUs, 2 = matrix cores) and, for batched systems,
   unit (particles per work unit) and split (force workgroups per unit).  Fixed rules
   give a plan for every cutoff; plans measured faster by the project's tuner
   (paper_1406_4254_amd/tune.py) are kept in a table keyed by (batched, nmax, lmax,
   precision, basis) and the particle count tuned at, and used for calls within a factor of 8 of that count.  Every tuned value is checked against
   the kernel's limits; an invalid one falls back to the fixed rules.  The table is
   read on first use from $ETICS_TUNING_FILE, else from etics_tuning.json next to
   libetics.so (if present).  Workspace sizes follow the plan in force when they are
   queried: change the table before sizing workspaces.  The table is process-wide and
   guarded by a lock. */

/* Replace the table with the plans of a JSON file ({"plans": [{"batched": 0, "nmax": ..,
   "lmax": .., "prec": .., "basis": .., "n": .., "nw": .., "tp": .., "streams": ..,
   "grid_mult": .., "unit": .., "split": .., "phase2": ..}, ...]}; a missing or 0
   parameter keeps the fixed rule's value).  Returns the number of plans read, or ETICS_EINVAL if the file
   cannot be read or parsed (the table is then unchanged). */
int etics_tuning_load(const char* path);

/* Add or replace one plan; params = {nw, tp, streams, grid_mult, unit, split, phase2}
   (nparams = 7; 0 keeps the fixed rule's value). */
int etics_tuning_set(int batched, int nmax, int lmax, int precision, int basis, int64_t n,
                     const int* params, int nparams);

/* Empty the table (fixed rules only); the file is not read afterwards. */
int etics_tuning_clear(void);

/* The plan a coefficient call over n particles would use (batched: n = ntotal, basis
   ETICS_BASIS_HO): out[0..8] = {nw, tp, streams, grid_mult, unit, split, phase2, tuned
   (0/1), workgroups of a single-system launch}.  nout >= 9. */
int etics_plan_info(int batched, int64_t n, int nmax, int lmax, int precision, int basis, int* out,
                    int nout);

/* Message describing the last non-zero return on the calling thread ("" if none). */
const char* etics_last_error(void);

/* Library version string. */
const char* etics_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ETICS_H */

/*
 * libhmc: the data-parallel hot path of Nf=2 Wilson-fermion Hybrid Monte
 * Carlo on one AMD MI355X (gfx950), as a C ABI.
 *
 * The operations are the ones the paper (Winter, "Gauge Field Generation on
 * Large-Scale GPU-Enabled Systems", Lattice 2012) lists for an HMC that runs
 * entirely on the accelerator (Sec. 1): pseudofermion refresh, momentum
 * update, force terms, projection of fields, reunitarisation of SU(3)
 * matrices, random numbers, exponentiation of SU(3) matrices, the fermion
 * matrix inversion, and the global sums sum/sumMulti.  The paper prints no
 * formula for any of them; each entry below states the textbook definition
 * it computes.
 *
 * Conventions (shared by every entry point):
 *   - Lattice L = {Lx, Ly, Lz, Lt}, every extent even and >= 2.  Site
 *     i = x + Lx*(y + Ly*(z + Lz*t)), parity (x+y+z+t) mod 2, checkerboard
 *     index s = i >> 1 within its parity; Vh = V/2 sites per parity.
 *   - Wilson operator M = 1 - kappa*D with the hopping term
 *       (D psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
 *                           + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)],
 *     gamma matrices in the DeGrand-Rossi basis (mu = 0..3 <-> x,y,z,t), and
 *     a factor -1 on every hop across the t = Lt-1 <-> 0 boundary
 *     (antiperiodic fermions; links are periodic).  D^dag = gamma5 D gamma5.
 *     Even/odd: Mhat = 1 - kappa^2 D_eo D_oe on even sites, det M = det Mhat.
 *   - Gauge action S_g = beta * sum_{x,mu<nu} (1 - Re Tr U_munu(x)/3);
 *     plaquette = sum Re Tr U_munu / (18 V).
 *   - Momenta P_mu(x) traceless Hermitian, T^a = lambda^a/2, kinetic term
 *     sum Tr P^2, equations of motion U' = i P U, P' = -F with
 *     F = sum_a T^a d/dt S(exp(i t T^a) U)|_0.
 *   - Fermion action S_f = phi_e^dag (Mhat^dag Mhat)^-1 phi_e.
 *   - Random numbers: Philox4x64-10 with counter (block, site i, stream,
 *     epoch) and key (seed, 0); uniform u = ((w >> 11) + 0.5) * 2^-53;
 *     Box-Muller on consecutive word pairs.  Streams: 0 weak-field start,
 *     1 momenta, 2 pseudofermion noise, 3 Metropolis, 4 sources.
 *
 * Memory: the caller owns every byte of device memory.  Device pointers are
 * plain addresses (e.g. torch tensors' data_ptr()); the library never calls
 * hipMalloc.  A fields object lives in one caller-provided device arena of
 * hmc_fields_bytes() bytes; its host metadata is freed by hmc_free_fields.
 *
 * Device field layouts (structure of arrays, component-major so that
 * consecutive sites are consecutive addresses):
 *   half spinor  [12 = spin*3+colour][Vh] complex, element type per prec:
 *                F64 double2, F32 float2, BF16 2 x bfloat16, F16 __half2
 *                followed by one float scale per site (components divided
 *                by the site's largest |re|,|im|)
 *   full spinor  two half spinors, even parity first
 *   gauge        [mu][parity][9 = row*3+col][Vh] complex
 *   momenta      [mu][parity][8][Vh] double: (P00, P11, Re P01, Im P01,
 *                Re P02, Im P02, Re P12, Im P12), P22 = -P00-P11
 * Canonical layouts (import/export; complex128, device memory):
 *   gauge / momenta [V][4][3][3], spinor [V][4][3].
 *
 * Streams: `stream` is a hipStream_t (0 = null stream).  Calls are
 * asynchronous on it, except those that return host values (stated per
 * entry), which synchronise that stream before returning.
 *
 * Errors: every entry returns an hmc_status; on failure
 * hmc_last_error() (thread-local) describes it.  No C++ exception crosses
 * this interface.
 */
#ifndef HMC_H
#define HMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hmc_status;
#define HMC_OK 0
#define HMC_E_ARG (-1)    /* invalid argument (null pointer, odd extent, size) */
#define HMC_E_OOM (-2)    /* arena too small, or a request can never fit */
#define HMC_E_HIP (-3)    /* a HIP runtime call failed */
#define HMC_E_NOCONV (-4) /* solver reached maxiter before the tolerance */
#define HMC_E_BUSY (-5)   /* poll: request not finished yet */
#define HMC_E_NAN (-6)    /* non-finite residual or energy change; trajectory rejected */

typedef enum { HMC_F64 = 0, HMC_F32 = 1, HMC_F16 = 2, HMC_BF16 = 3 } hmc_prec;

typedef enum {
  HMC_KIND_HALF_SPINOR = 0,
  HMC_KIND_FULL_SPINOR = 1,
  HMC_KIND_GAUGE = 2,
  HMC_KIND_MOMENTA = 3
} hmc_kind;

typedef struct {
  int32_t L[4];
} hmc_geom;

typedef struct {
  double beta;  /* gauge coupling */
  double kappa; /* hopping parameter */
} hmc_action;

typedef struct hmc_fields hmc_fields;

/* Thread-local description of the last failure on this thread. */
const char* hmc_last_error(void);
/* Library version (major, minor). */
hmc_status hmc_get_version(int32_t* major, int32_t* minor);

/* Bytes of one device field of the given kind and storage precision
 * (momenta exist in F64 only): one entry per lattice site and component,
 * the site-per-thread data of Sec. 3 (Tab. 1: outer x spin x colour x
 * reality).  HMC_E_ARG on bad geometry. */
hmc_status hmc_field_bytes(const hmc_geom* geom, hmc_prec prec, hmc_kind kind, size_t* bytes);

/* Flags of hmc_alloc_fields. */
#define HMC_FIELDS_LOWPREC 1u /* also hold F32/F16/BF16 link copies and inner solver vectors */

/* Arena bytes hmc_alloc_fields needs for this geometry and flags (all
 * fields of a trajectory stay resident in HBM: the caller's arena takes
 * the place of the automatic memory management of Sec. 5). */
hmc_status hmc_fields_bytes(const hmc_geom* geom, uint32_t flags, size_t* bytes);

/* Create a fields object inside the caller's device arena (at least
 * hmc_fields_bytes bytes, 256-byte aligned): the lattice fields of the HMC
 * (Sec. 1) laid out one site per work-item (Sec. 3, Tab. 1), resident for
 * the object's lifetime (no spilling, unlike Sec. 5).  It holds: the gauge field U,
 * its backup, the momenta P, the pseudofermion noise eta_e and phi_e, the
 * solution X_e, the force vectors and the solver work space.  Nothing is
 * initialised: import or generate U before use.  The arena must outlive
 * the object.  HMC_E_ARG on bad geometry or null pointers, HMC_E_OOM when
 * arena_bytes is too small. */
hmc_status hmc_alloc_fields(const hmc_geom* geom, const hmc_action* action, uint32_t flags, void* arena,
                            size_t arena_bytes, hmc_fields** out);
/* Release the host metadata (the arena stays the caller's; Sec. 5's
 * memory manager has no counterpart here). */
hmc_status hmc_free_fields(hmc_fields* f);
/* Change beta and kappa of an existing fields object. */
hmc_status hmc_set_action(hmc_fields* f, const hmc_action* action);

/* Internal fields a caller may read or write directly (device pointers in
 * the layouts above, F64). */
typedef enum {
  HMC_FIELD_GAUGE = 0,
  HMC_FIELD_MOMENTA = 1,
  HMC_FIELD_ETA = 2, /* even half spinor */
  HMC_FIELD_PHI = 3, /* even half spinor */
  HMC_FIELD_XE = 4   /* even half spinor: last solve of the fermion force */
} hmc_field_id;
hmc_status hmc_field_pointer(hmc_fields* f, hmc_field_id which, void** ptr);
/* Writing U through the HMC_FIELD_GAUGE pointer: call hmc_sync_lowprec
 * afterwards.  Fetching that pointer switches the hopping kernels to
 * full-link loads until then (see hmc_links_two_row). */

/* Canonical <-> device layout conversion (both buffers in device memory):
 * site-major canonical arrays <-> the component-major structure of arrays
 * in which consecutive work-items read consecutive addresses (the
 * site-per-thread mapping of Sec. 3 with the coalesced layout Sec. 9 names
 * as future work).
 * Spinors: `parity` 0 or 1 converts one half spinor (export writes zeros on
 * the other parity's sites of the canonical buffer); -1 converts a full
 * spinor.  Gauge/momenta act on the fields object's U / P.  The canonical
 * momenta must be traceless Hermitian (the compact form keeps P00, P11 and
 * the upper triangle). */
hmc_status hmc_import_gauge(hmc_fields* f, const void* canon, void* stream);
hmc_status hmc_export_gauge(hmc_fields* f, void* canon, void* stream);
hmc_status hmc_import_momenta(hmc_fields* f, const void* canon, void* stream);
hmc_status hmc_export_momenta(hmc_fields* f, void* canon, void* stream);
hmc_status hmc_import_spinor(hmc_fields* f, void* dst, const void* canon, int32_t parity, void* stream);
hmc_status hmc_export_spinor(hmc_fields* f, void* canon, const void* src, int32_t parity, void* stream);

/* Convert a half spinor between storage precisions (F64 <-> F32/F16/BF16). */
hmc_status hmc_convert_spinor(hmc_fields* f, void* dst, hmc_prec dst_prec, const void* src, hmc_prec src_prec,
                              void* stream);
/* Re-derive everything the library keeps about U after U was written in
 * place: checks whether every link is SU(3) to 1e-14 (rows 0 and 1
 * orthonormal, row 2 = conj(row0 x row1); then the hopping and staple
 * kernels read a compact form of each link and rebuild the rest; one
 * reduction, synchronises the stream) and, with HMC_FIELDS_LOWPREC,
 * refreshes the F32/F16/BF16 link copies (hmc_cg_solve refreshes those
 * itself when the library changed U). */
hmc_status hmc_sync_lowprec(hmc_fields* f, void* stream);
/* *on = 1 if the kernels read a compact form of each link, else 0 (all
 * nine entries are read).  Compact forms need U to be SU(3) to rounding:
 * set by hmc_weak_field_start, hmc_exp_update_reunit and the integrator,
 * which reunitarise, and by the check in hmc_import_gauge /
 * hmc_sync_lowprec.  The forms: rows 0 and 1, rebuilding row 2 as
 * conj(row0 x row1) (2/3 of the link bytes), or row 0 and column 2,
 * rebuilding u10, u11 from orthogonality and det = 1 and then row 2 (5/9 of
 * the link bytes; links with |u02|^2 > 15/16 read u10, u11); which one per
 * lattice and kernel family: hmc_tune_query.  Every form gives the same
 * operator on SU(3) fields up to rounding. */
hmc_status hmc_links_two_row(hmc_fields* f, int32_t* on);

/* One half-lattice hop of the fermion matrix whose inversion takes most
 * of the floating-point work (Sec. 1): out = D_{p <- 1-p} in (dagger:
 * D^dag), p = out_parity.  in/out are half spinors of storage `prec`; links come from U
 * (F64) or its low-precision copy.  Arithmetic is FP64 for F64, else FP32. */
hmc_status hmc_wilson_dslash(hmc_fields* f, void* out, const void* in, int32_t out_parity, int32_t dagger,
                             hmc_prec prec, void* stream);
/* The even-odd preconditioned fermion matrix (Sec. 1, fermion matrix):
 * out_e = Mhat in_e (dagger: Mhat^dag), half spinors of storage `prec`. */
hmc_status hmc_mhat(hmc_fields* f, void* out, const void* in, int32_t dagger, hmc_prec prec, void* stream);
/* Full Wilson fermion matrix (Sec. 1) on full F64 spinors: out = M in
 * (dagger: M^dag). */
hmc_status hmc_wilson_m(hmc_fields* f, void* out, const void* in, int32_t dagger, void* stream);

/* Global sums (QDP++ sum / innerProduct / sumMulti, Sec. 1), deterministic:
 * per-block partials in a fixed order, then one fixed-order pass.  Each
 * synchronises the stream and returns host values.  `nhalves` = 1 (half
 * spinor) or 2 (full spinor).
 *   hmc_norm2: sum |x|^2 (x of storage prec).
 *   hmc_inner: <a, b> = sum conj(a) b (F64), out[0] = Re, out[1] = Im.
 *   hmc_sum_multi: out[k] = sum of |x(site)|^2 over the sites with
 *     subset[site] == k; subset is an int32 device array in the field's own
 *     site order ([parity][Vh]; for nhalves = 1 only the first Vh entries),
 *     values in [0, nsub) (other values are ignored).  nsub <= 1024. */
hmc_status hmc_norm2(hmc_fields* f, const void* x, int32_t nhalves, hmc_prec prec, double* out, void* stream);
hmc_status hmc_inner(hmc_fields* f, const void* a, const void* b, int32_t nhalves, double* out, void* stream);
hmc_status hmc_sum_multi(hmc_fields* f, const void* x, int32_t nhalves, const int32_t* subset, int32_t nsub,
                         double* out, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hmc_norm2
 * on a spinor of lattice `geom` (layout and storage as in hmc_norm2)
 * without a fields object.  The block partial sums go to a static device
 * array of 4096 doubles (32 KiB) that the library holds on each GPU it runs
 * on until the process ends; the call allocates nothing, reads nothing back
 * and writes the sum to the device double out_dev.  Asynchronous on the
 * stream.  The result is bit-identical to hmc_norm2's.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (different
 * streams, or threads without ordering) race; serialise them, e.g. on one
 * stream.  HMC_E_ARG on bad geometry or arguments, or when the partial
 * sums (two halves x up to 2048 blocks) would exceed the array. */
hmc_status hmc_norm2_static(const hmc_geom* geom, const void* x, int32_t nhalves, hmc_prec prec, double* out_dev,
                            void* stream);

/* Plaquette (1/18V) sum Re Tr U_munu, gauge action S_g and kinetic term
 * sum Tr P^2 of the fields object: the gauge and momentum parts of the HMC
 * Hamiltonian (Sec. 1), each a global sum (Sec. 1, sum); synchronise and
 * return host values. */
hmc_status hmc_plaquette(hmc_fields* f, double* out, void* stream);
hmc_status hmc_gauge_action(hmc_fields* f, double* out, void* stream);
hmc_status hmc_kinetic_energy(hmc_fields* f, double* out, void* stream);

/* Momentum update with the gauge force (Sec. 1 "force term", "momentum
 * update"): P <- P - coef * F_g with
 *   F_g = -(i beta/12) [(W - W^dag) - Tr(W - W^dag)/3],  W = U_mu(x) A_mu(x),
 * A_mu the sum of the six staples. */
hmc_status hmc_gauge_force(hmc_fields* f, double coef, void* stream);

/* Momentum update with the fermion force (Sec. 1 "force term", "momentum
 * update") of S_f for the solution X_e =
 * (Mhat^dag Mhat)^-1 phi_e (even half spinor, F64): the library forms
 * X_o = D_oe X_e, Y_e = Mhat X_e, Y_o = (D^dag)_oe Y_e and applies
 *   P <- P - coef * (i kappa^2/2) [(W - W^dag) - Tr(W - W^dag)/3],
 *   W = U_mu(x) M1 - M2 U_mu(x)^dag,
 *   M1 = s tr_spin[(1 - gamma_mu) X(x+mu) Y(x)^dag],
 *   M2 = s tr_spin[(1 + gamma_mu) X(x) Y(x+mu)^dag],
 * s the time-boundary sign of the hop x -> x+mu. */
hmc_status hmc_fermion_force(hmc_fields* f, const void* X_e, double coef, void* stream);

/* Link update of the integrator with exponentiation and reunitarisation
 * (Sec. 1): U_mu(x) <- reunit(exp(i eps P_mu(x)) U_mu(x)); reunit is the
 * row Gram-Schmidt projection (row 2 = conj(row0 x row1)). */
hmc_status hmc_exp_update_reunit(hmc_fields* f, double eps, void* stream);

/* Refresh (Sec. 1 "pseudofermion refresh", "random number generator"):
 *   HMC_REFRESH_MOM: P_mu(x) = sum_a w_a T^a, w ~ N(0,1) from stream 1 at
 *     epoch traj; Gaussian index mu*8 + (a-1).
 *   HMC_REFRESH_PF: eta_e complex Gaussian with E|eta|^2 = 1 (stream 2,
 *     epoch traj, components (spin, colour, re/im)), phi_e = Mhat^dag eta_e. */
#define HMC_REFRESH_MOM 1u
#define HMC_REFRESH_PF 2u
hmc_status hmc_refresh(hmc_fields* f, uint64_t seed, uint64_t traj, uint32_t what, void* stream);

/* Weak-field start from the generator, exponentiation and
 * reunitarisation of Sec. 1: U_mu(x) = reunit(exp(i eps H_mu(x))),
 * H = sum_a h_a T^a, h ~ N(0,1) from stream 0, epoch 0. */
hmc_status hmc_weak_field_start(hmc_fields* f, uint64_t seed, double eps, void* stream);

/* Solver source (right-hand side of a fermion-matrix inversion, Sec. 1;
 * noise from the generator of Sec. 1) on a full F64 spinor b (stream 4,
 * epoch = source index):
 * HMC_SOURCE_GAUSS unit-variance Gaussian per real component;
 * HMC_SOURCE_Z2 (+-1 +-i)/sqrt2 with signs from bit 63 of successive words;
 * HMC_SOURCE_POINT 1 at site 0, spin 0, colour 0. */
#define HMC_SOURCE_GAUSS 0
#define HMC_SOURCE_Z2 1
#define HMC_SOURCE_POINT 2
hmc_status hmc_make_source(hmc_fields* f, void* b, int32_t kind, uint64_t seed, uint64_t epoch, void* stream);

/* Raw generator access for bit-exactness checks: for each lexicographic
 * site in sites[0..nsites) (int64, device) write nblocks Philox blocks
 * (4 words each) to out[site_k][nblocks*4] (device, uint64), or n
 * Box-Muller Gaussians to out[site_k][n] (device, double, n even <= 32). */
hmc_status hmc_random_words(uint64_t seed, uint64_t rng_stream, uint64_t epoch, const int64_t* sites,
                            int32_t nsites, int32_t nblocks, uint64_t* out, void* stream);
hmc_status hmc_random_gaussians(uint64_t seed, uint64_t rng_stream, uint64_t epoch, const int64_t* sites,
                                int32_t nsites, int32_t n, double* out, void* stream);

/* Krylov solve (the "fermion matrix inversion" of Sec. 1).
 *   HMC_CG_NORMAL_MHAT: x_e = (Mhat^dag Mhat)^-1 b_e by conjugate gradient
 *     from x = 0, stopping at the first k with |r_k| <= tol |b| (recursive
 *     residual).  x, b: even half spinors F64.
 *   HMC_CG_WILSON_SOLVE: M x = b for full F64 spinors through the Schur
 *     complement: bhat_e = b_e + kappa D_eo b_o, CGLS on Mhat x_e = bhat_e
 *     until |bhat_e - Mhat x_e| <= tol |b|, x_o = b_o + kappa D_oe x_e.
 * prec = HMC_F64 runs FP64 throughout.  F32 / F16 / BF16 run the inner
 * iteration on vectors and links stored in that format with FP32
 * arithmetic and FP64 global sums, and replace the residual by the FP64
 * true residual b - A x whenever the inner residual fell by
 * reliable_delta (Clark et al., Comput. Phys. Commun. 181 (2010) 1517),
 * and at least every 48 inner iterations; an update keeps the search
 * direction unless the FP64 residual exceeds twice the inner one or did
 * not fall since the previous update, when it restarts it from the new
 * residual (BF16 storage with delta <= 0.01 needs this); the exit test is
 * always on the FP64 true residual.  Needs HMC_FIELDS_LOWPREC.
 * fixed_iters > 0 (F64 only) runs exactly that many iterations and ignores
 * tol.  Synchronises the stream; fills stats.  HMC_E_NOCONV when maxiter
 * is reached (after exactly maxiter iterations; x holds the last iterate);
 * HMC_E_NAN when |b|^2 or a residual norm is not finite (the iteration
 * stops at the first such norm; x holds the last iterate). */
typedef enum { HMC_CG_NORMAL_MHAT = 0, HMC_CG_WILSON_SOLVE = 1 } hmc_cg_mode;
typedef struct {
  double tol;
  int32_t maxiter;
  int32_t mode;   /* hmc_cg_mode */
  int32_t prec;   /* hmc_prec of the inner iteration */
  int32_t fixed_iters;
  double reliable_delta; /* <= 0 selects 0.01 for F32, 0.1 for F16 / BF16 */
  int32_t initial_guess; /* CG on Mhat^dag Mhat only: != 0 starts from the x passed in
                            (r0 = b - A x0); 0 starts from x0 = 0 */
  int32_t pad;
} hmc_cg_params;
typedef struct {
  int32_t iters;            /* total (inner) iterations */
  int32_t reliable_updates; /* FP64 residual replacements */
  double rel_res;           /* last recursive residual / |b| */
  double true_rel_res;      /* FP64 |b - A x| / |b| (full M for Wilson solves) */
  double seconds;           /* wall time of the solve */
} hmc_cg_stats;
hmc_status hmc_cg_solve(hmc_fields* f, void* x, const void* b, const hmc_cg_params* params, hmc_cg_stats* stats,
                        void* stream);

/* Leapfrog molecular dynamics (the HMC integration of Sec. 1: momentum
 * updates with the force terms, link updates by exponentiation and
 * reunitarisation), PQP: with eps = tau/nsteps,
 *   P -= (eps/2) F(U); then nsteps times { U <- reunit(exp(i eps P) U);
 *   P -= eps_k F(U) } with eps_k = eps except eps/2 for the last step;
 * F = F_g + F_f, the fermion force from a CG solve of phi_e (FP64).
 * tau may be negative.  X_e holds the last solve.  Synchronises.  The
 * integration always runs to the end; then HMC_E_NAN if a solve met a
 * non-finite residual, else HMC_E_NOCONV if a solve stopped at maxiter. */
typedef struct {
  int32_t solves;
  int32_t iters_total;
  int32_t iters_max;
  int32_t nonconverged; /* solves that did not reach tol (non-finite ones included) */
  int32_t nonfinite;    /* solves whose residual became non-finite */
} hmc_md_stats;
hmc_status hmc_md_leapfrog(hmc_fields* f, double tau, int32_t nsteps, const hmc_cg_params* cg, hmc_md_stats* stats,
                           void* stream);

/* One HMC trajectory with index traj (Sec. 1's HMC; Sec. 7's gauge field
 * generation): backup U; refresh momenta and pseudofermions; H_old = sum
 * Tr P^2 + S_g + eta^dag eta; leapfrog; H_new = sum Tr P^2 + S_g +
 * phi^dag X_e; accept iff dH <= 0 or u < exp(-dH), u from stream 3 at epoch
 * traj (site 0, block 0, word 0); restore U on reject.  Failures force a
 * reject (U restored bit for bit from the backup) and fill the result:
 * a non-finite dH, or a solve that met a non-finite residual, returns
 * HMC_E_NAN; otherwise a solve that stopped at maxiter returns
 * HMC_E_NOCONV.  HMC_E_NAN takes precedence because a non-finite field
 * also stops every solve that reads it.  Synchronises. */
typedef struct {
  double tau;
  int32_t nsteps;
  int32_t n_chrono; /* 0: every force solve starts from x0 = 0; 1..4: from the
                       chronological guess, the Galerkin projection of the
                       solve onto the span of the last n_chrono solutions of
                       the same trajectory (Brower et al., Nucl. Phys. B 484
                       (1997) 353) */
  hmc_cg_params cg;
} hmc_traj_params;
typedef struct {
  double H_old, H_new, dH;
  double S_g_old, S_g_new, S_f_old, S_f_new, KE_old, KE_new;
  double plaquette; /* after accept/reject */
  double u;         /* Metropolis uniform */
  int32_t accepted;
  int32_t cg_iters_total;
  int32_t cg_iters_max;
  int32_t nonconverged;
  double seconds;
} hmc_traj_result;
hmc_status hmc_trajectory(hmc_fields* f, uint64_t seed, uint64_t traj, const hmc_traj_params* params,
                          hmc_traj_result* result, void* stream);

/* STREAM triad a = b + s c over n doubles (n even; device buffers, 16-byte
 * aligned, a distinct from b and c), with non-temporal loads and stores
 * when nontemporal != 0: the attainable streaming rate for the access
 * pattern of the field kernels (16-byte lanes), against which their
 * bandwidth is read.  Asynchronous on the stream. */
hmc_status hmc_stream_triad(void* a, const void* b, const void* c, double s, uint64_t n, int32_t nontemporal,
                            void* stream);

/* ---- Launch auto-tuning (the auto-tuner of Sec. 4, for the launch shapes
 * and link forms this library offers).  Kinds:
 *   HMC_TUNE_DSLASH (per storage precision): 1 = one site per work-item,
 *     2 / 4 = direction split with that many wavefronts per 64-site group;
 *   HMC_TUNE_GAUGE_FORCE (prec HMC_F64): 0 = one link per work-item,
 *     direction by direction; 1 = plane split; 2 = a block per 64 sites and
 *     all four directions, in the tiled walk of the Dslash where the lattice
 *     admits it (y-blocks of two chunks, or the chunks of the t-slices where
 *     a z-plane is not a whole number of chunks), else linearly (the
 *     plaquette sum and the fermion force always walk this way);
 *   HMC_TUNE_DSLASH_LINKS (per storage precision): reals read per SU(3)
 *     link by the hopping kernels, 12 = rows 0 and 1, 10 = row 0 and
 *     column 2 (the fermion force follows the FP64 entry);
 *   HMC_TUNE_GAUGE_FORCE_LINKS (prec HMC_F64): the same for the staple
 *     force (the plaquette sum on SU(3) links reads two rows, measured
 *     fastest there; on other links all nine entries);
 *   HMC_TUNE_DSLASH_STREAM (per storage precision): 1 = the Dslash reads its
 *     compact links and writes its output with non-temporal hints;
 *   HMC_TUNE_DSLASH_ORDER (per storage precision): 1 = the one-site-per-
 *     work-item Dslash walks each XCD's t-slices z-plane by z-plane, t-slice
 *     by t-slice, so neighbour spinors are reused in that XCD's L2 (lattices
 *     with L3 a multiple of 8, Vh a multiple of 2048 and L0 L1 / 2 a
 *     multiple of 64; where only L0 L1 L2 / 2 is, the walk takes the 64-site
 *     chunks of the t-slices, t-slice fastest); n >= 2 = the z-plane walk
 *     over y-blocks of n 64-site chunks of each z-plane in turn, so several
 *     z-planes are in flight at once (n divides L0 L1 / 128, n <= 64; any
 *     other n reads as 1);
 *   HMC_TUNE_DSLASH_OCC (per storage precision): workgroups per CU of the
 *     tiled order, 2 = at most two (an unused LDS reservation keeps the
 *     wavefronts in flight close together in the walk), 0 = as many as
 *     registers allow.
 * Decision order: environment override (HMC_DSLASH_SPLIT, HMC_GFORCE_PLANES
 * = 0 / 1 / 2, HMC_LINK_FORM = 18 / 12 / 10, HMC_LINK_STREAM = 0 / 1,
 * HMC_DSLASH_ORDER = 0 / 1 / n, HMC_DSLASH_OCC = 0 / 2) > table entry for
 * the lattice extents > built-in rule.
 * HMC_TUNE_DB names a table file read on first use.  Table file: text lines
 * "kind L0 L1 L2 L3 prec choice us" with kind dslash, gauge_force,
 * dslash_links, gauge_force_links, dslash_stream, dslash_order or
 * dslash_occupancy ('#' lines and malformed lines are ignored).  Shapes are
 * fixed per solve (and per service request) when it starts; do not tune
 * while solves or a service run on the same lattice extents. */
typedef enum {
  HMC_TUNE_DSLASH = 0,
  HMC_TUNE_GAUGE_FORCE = 1,
  HMC_TUNE_DSLASH_LINKS = 2,
  HMC_TUNE_GAUGE_FORCE_LINKS = 3,
  HMC_TUNE_DSLASH_STREAM = 4,
  HMC_TUNE_DSLASH_ORDER = 5,
  HMC_TUNE_DSLASH_OCC = 6
} hmc_tune_kind;
/* Times every candidate on f's lattice and stores the fastest in the
 * table: for each storage precision the Dslash shape x link form pairs
 * (then streaming, and the site orders x workgroups per CU, for the best
 * pair)
 * where it runs, inside a solve (CG on Mhat^dag Mhat from Gaussian noise to
 * 1e-10 or 100 iterations: FP64 CG, and with HMC_FIELDS_LOWPREC
 * mixed-precision CG with that storage inside; "us" = microseconds per
 * iteration); the staple force's shape x link form per launch with coef 0
 * (P unchanged).  Link forms are tuned only when U is SU(3) (see
 * hmc_links_two_row).  With db_path != NULL the table is merged into that
 * file.  Overwrites f's eta, X_e and solver work vectors.  HMC_E_ARG when
 * an environment override is set.  Synchronises. */
hmc_status hmc_autotune(hmc_fields* f, const char* db_path, void* stream);
hmc_status hmc_tune_load(const char* path, int32_t* n_entries);
hmc_status hmc_tune_save(const char* path, int32_t* n_entries);
/* Active decision for lattice L (*tuned = 1 when it comes from the table). */
hmc_status hmc_tune_query(const int32_t* L, int32_t kind, int32_t prec, int32_t* choice, int32_t* tuned);

/* ---- Mass-preconditioned (Hasenbusch) two-flavour HMC on nested time
 * scales (the production setup of Sec. 7).  det(A) is split with a heavier
 * hopping parameter kappa_h (0 < kappa_h <= kappa), A = Mhat^dag Mhat:
 *   S_1 = phi_1^dag A_h^-1 phi_1,             phi_1 = Mhat_h^dag eta_1,
 *   S_2 = chi^dag A^-1 chi, chi = Mhat_h^dag phi_2,
 *                                             phi_2 = Mhat_h A_h^-1 Mhat^dag eta_2,
 * eta_1 from Philox stream 2, eta_2 from stream 5 (epoch traj, even
 * sites).  Forces: S_1 is the Wilson force at kappa_h; S_2 is the Wilson
 * bilinear of (X_2, Mhat X_2) at kappa minus that of (X_2, phi_2) at
 * kappa_h, X_2 = A^-1 chi.  Integrator: nested PQP leapfrog, ratio
 * monomial on the outer scale (n_ratio steps over tau), the heavy monomial
 * n_heavy steps per outer step, the gauge force n_gauge steps per heavy
 * step; kicks that fall between the same two link updates are applied
 * together, ratio then heavy then gauge.  Force evaluations per
 * trajectory: n_ratio + 1 ratio solves, n_ratio n_heavy + 1 heavy solves,
 * n_ratio n_heavy n_gauge + 1 gauge forces. */
typedef struct {
  double tau;
  double kappa_h;
  int32_t n_ratio, n_heavy, n_gauge;
  int32_t pad;
  hmc_cg_params cg; /* both monomials (mode ignored: CG on A) */
} hmc_mts_params;
typedef struct {
  double S1_old, S2_old, S1_new, S2_new;
  int32_t solves_ratio, solves_heavy, gauge_forces, link_updates;
  int32_t iters_ratio, iters_heavy, nonconverged, nonfinite;
} hmc_mts_stats;
/* P -= coef F for the Wilson-force bilinear of X = (X_e, D_oe X_e) and
 * Y = (Y_e, (D^dag)_oe Y_e) at hopping parameter kappa_c (the plain
 * monomial is Y_e = Mhat X_e at kappa_c = kappa).  X_e, Y_e: even F64 half
 * spinors. */
hmc_status hmc_fermion_force_bilinear(hmc_fields* f, const void* X_e, const void* Y_e, double kappa_c, double coef,
                                      void* stream);
/* Integrate U and P over p->tau with the nested schedule; phi_1 is the
 * fields' HMC_FIELD_PHI, phi_2 the given even half spinor.  tau may be
 * negative.  Synchronises; fills *stats (actions left 0). */
hmc_status hmc_md_mts(hmc_fields* f, const void* phi2, const hmc_mts_params* p, hmc_mts_stats* stats,
                      void* stream);
/* One mass-preconditioned trajectory; H = sum Tr P^2 + S_g + S_1 + S_2,
 * accept/reject and return codes as hmc_trajectory. */
hmc_status hmc_trajectory_mts(hmc_fields* f, uint64_t seed, uint64_t traj, const hmc_mts_params* p,
                              hmc_traj_result* result, hmc_mts_stats* stats, void* stream);

/* Solve service: continuous batching of Wilson solves M x = b (the
 * fermion-matrix inversions of Sec. 1 as a request stream).  Each request
 * brings its own lattice volume, kappa, weak-field gauge field (drawn on the
 * device from its seed) and source.  A scheduler admits requests in FIFO
 * order whenever their device footprint (hmc_request_bytes) fits into the
 * free part of the caller's arena, keeps each request's gauge field and
 * solver state resident, and advances all admitted requests of the same
 * volume together: every solver step is one launch over the whole group
 * (blockIdx.y = request).  Requests that arrive while others run join at
 * the next round; finished ones leave and free their memory.  The solver is
 * CGLS with reliable updates (HMC_CG_WILSON_SOLVE semantics) with inner
 * storage `inner_prec`, exit on the FP64 true residual; each request's
 * arithmetic depends only on its own data, so its result is the same alone
 * and in any mix.
 *
 * With manual = 0 a scheduler thread runs rounds while work is pending;
 * with manual = 1 progress happens only in hmc_service_step (deterministic
 * tests).  The caller owns the streams as it owns the memory (Sec. 5.1:
 * work asynchronous on streams): the k-th volume group in use runs on
 * streams[k mod n_streams], so n_streams > 1 lets different volumes
 * overlap on the device; the library creates and destroys no stream, and
 * the streams must outlive the service.  Times are seconds since
 * hmc_service_create. */
#define HMC_SERVICE_MAX_STREAMS 8
typedef struct {
  void* arena;            /* device memory owned by the caller */
  size_t arena_bytes;
  int32_t max_batch;      /* max requests advanced together per volume (<= 256) */
  int32_t inner_prec;     /* hmc_prec of the inner iteration */
  double tol;             /* |b - M x| <= tol |b| */
  int32_t maxiter;        /* inner iterations per request */
  int32_t manual;
  int32_t chunk;          /* iterations per round (<= 0 selects 16) */
  int32_t n_streams;      /* 1..HMC_SERVICE_MAX_STREAMS entries of streams[] used */
  void* streams[HMC_SERVICE_MAX_STREAMS]; /* hipStream_t of the caller (0 = null stream) */
  double reliable_delta;  /* as in hmc_cg_params (<= 0: 0.01 for F32, 0.1 for F16 / BF16) */
} hmc_service_params;
typedef struct {
  int32_t L[4];
  double kappa;
  uint64_t gauge_seed;
  double gauge_eps;
  int32_t source_kind; /* HMC_SOURCE_* */
  int32_t pad;
  uint64_t source_seed;
  uint64_t source_epoch;
  void* out; /* optional device buffer (full F64 spinor of this volume) for x */
} hmc_solve_request;
typedef struct {
  int32_t status; /* HMC_OK, HMC_E_NOCONV, HMC_E_OOM */
  int32_t iters;
  int32_t reliable_updates;
  int32_t max_group; /* largest group this request was advanced in */
  double true_rel_res;
  double t_submit, t_start, t_done;
} hmc_solve_result;
typedef struct hmc_service hmc_service;

/* Device bytes one request occupies in the service arena: its gauge
 * field, source, solution and solver vectors, resident while it runs
 * (the admission footprint; no spilling as in Sec. 5). */
hmc_status hmc_request_bytes(const hmc_solve_request* req, int32_t inner_prec, size_t* bytes);
/* Start a service on the caller's arena and streams (Sec. 5.1: device work
 * asynchronous on streams, host progress alongside).  HMC_E_ARG on bad
 * parameters, HMC_E_OOM if the arena cannot hold the service header. */
hmc_status hmc_service_create(const hmc_service_params* params, hmc_service** out);
/* Submit one Wilson solve (a fermion-matrix inversion, Sec. 1).
 * Non-blocking.  HMC_E_OOM if the request can never fit the arena,
 * HMC_E_ARG on a bad request; otherwise it waits for memory. */
hmc_status hmc_service_submit(hmc_service* svc, const hmc_solve_request* req, uint64_t* ticket);
/* Poll a request without blocking (the host progresses beside the device,
 * Sec. 5.1).  HMC_E_BUSY until the request has finished; then fills res and
 * returns the request's status.  A finished ticket stays queryable. */
hmc_status hmc_service_poll(hmc_service* svc, uint64_t ticket, hmc_solve_result* res);
/* Blocks until the request has finished (runs rounds itself in manual
 * mode); the synchronising counterpart of the asynchronous calls of
 * Sec. 5.1. */
hmc_status hmc_service_wait(hmc_service* svc, uint64_t ticket, hmc_solve_result* res);
/* One scheduling round (admit, advance, retire: a batch of the Sec. 1
 * inversions advanced together); *pending = requests not yet finished.
 * Manual mode only. */
hmc_status hmc_service_step(hmc_service* svc, int32_t* pending);
/* Stops the scheduler (after the current round), waits for the caller's
 * streams (Sec. 5.1) and releases host state; unfinished requests are
 * dropped. */
hmc_status hmc_service_destroy(hmc_service* svc);

/* Kernel timing with HIP events on the launch streams (the measurement
 * behind the performance figures of Sec. 7).  With sample_every = n > 0
 * every n-th launch of each kernel family is bracketed by a pair of events
 * (up to a fixed pool; later launches go untimed); 0 disables.
 * hmc_timing_read synchronises the recorded events and returns, per family,
 * the number of timed launches, their summed milliseconds, their summed
 * bytes in two conventions, and the number of all launches (timed or not),
 * so that average x calls estimates the family's total time.  `bytes` are
 * the operation's algorithmic bytes: each datum it reads once, each output
 * written once, an SU(3) link as its nine complex entries (144 B in FP64),
 * a half spinor site as its twelve (192 B).  `bytes_moved` are the bytes
 * of what the kernel as implemented must move: on SU(3) fields the compact
 * links it reads (96 B for two rows, 80 B for row 0 and column 2).
 * Process-wide, not thread-safe against concurrent launches. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double bytes;       /* algorithmic */
  int64_t calls;      /* all launches of the family while timing was enabled */
  double bytes_moved; /* as implemented */
} hmc_timing_entry;
hmc_status hmc_timing_enable(int32_t sample_every);
hmc_status hmc_timing_reset(void);
hmc_status hmc_timing_read(hmc_timing_entry* out, int32_t max_entries, int32_t* n_entries);
/* Launches n empty one-wavefront kernels through the same kernel-stamped
 * event mechanism (family "other"): their timed duration is the floor that
 * the event pair adds to every timed launch. */
hmc_status hmc_timing_probe(int32_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HMC_H */

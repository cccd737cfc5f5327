/*
 * dloops.h -- C ABI of the MI355X (gfx950) library for disconnected quark
 * loops with N_f = 2 Wilson fermions, after Alexandrou, Christaras, O Cais and
 * Strelchenko, "Exact calculation of disconnected loops" (Lattice 2010).
 *
 * The method (Sections 2 and 3 of the paper): repeated Krylov inversions of
 * the Wilson-Dirac matrix M = 1 - kappa D_hop on diluted complex-Z2 noise
 * sources (or unit point sources, the exact method), followed by the local
 * zero-momentum loop traces
 *     L_Gamma(t) = sum_{x: x_4 = t} Tr[Gamma M^-1(x, x)],
 * estimated per noise vector as sum_d eta_d^+ P_t Gamma M^-1 eta_d, and the
 * truncated solver method's low/high-precision split.
 *
 * Conventions (the paper names Wilson fermions and a basis without writing
 * them down; these are the readings used):
 *   - dims = {X, Y, Z, T}, every extent even and >= 2; site index
 *     i = x + X*(y + Y*(z + Z*t));
 *   - canonical spinor field: complex128 [V][4 spin][3 colour], interleaved
 *     (re, im) doubles; n fields are contiguous, [n][V][4][3];
 *   - canonical gauge field: complex128 [4 mu][V][3][3], U_mu(x)_{ab};
 *   - chiral basis gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 =
 *     [[0, 1], [1, 0]], gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 =
 *     diag(1, 1, -1, -1); Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3 for
 *     n = n0 + 2 n1 + 4 n2 + 8 n3 (Gamma_0 = 1, Gamma_15 = gamma_5,
 *     Gamma_5 = gamma_1 gamma_3);
 *   - (D psi)(x) = sum_mu (1 - gamma_mu) b U_mu(x) psi(x + mu)
 *                      + (1 + gamma_mu) b U_mu(x - mu)^+ psi(x - mu),
 *     Wilson r = 1, b = -1 on hops across the time boundary when it is
 *     antiperiodic, +1 otherwise;
 *   - complex Z2 noise: entry (noise n, site i, spin s, colour c) is output
 *     number ((n*V + i)*4 + s)*3 + c of the SplitMix64 stream (Steele, Lea and
 *     Flood 2014) seeded with `seed`; bit 0 gives the sign of the real part and
 *     bit 1 that of the imaginary part (0 -> +), amplitude 1/sqrt(2);
 *   - dilution (Section 2) scheme bits: 1 = spin-colour (12 classes,
 *     d = 3 s + c), 16 = spin (4 classes, s), 32 = spin even-odd
 *     partitioning (2 classes, s & 1), 8 = colour (3 classes, c), 2 = cubic
 *     spatial (8 classes, (x&1) + 2(y&1) + 4(z&1)), 4 = spatial even-odd
 *     (2 classes, (x+y+z+t)&1); enabled factors combine in that order, the
 *     later factor running fastest (so 16 | 8 gives the classes of 1).  Bit 1
 *     excludes 8, 16 and 32; 16 and 32 exclude each other.  64 = time
 *     dilution: noise n is supported on timeslice n mod T only (no extra
 *     classes; its loops are zero on the other timeslices, and the noises
 *     cover the timeslices in turn).
 *
 * Every call returns a dl_status.  On failure dl_last_error() describes it
 * (thread-local text, valid until the next call on the same thread).
 * Arguments are validated before any device work; an invalid argument leaves
 * every output untouched.  No C++ exception crosses this interface.
 *
 * Pointers are borrowed.  "device" pointers are HIP device memory on the
 * current device (e.g. torch tensors' data_ptr()); "host" pointers are host
 * memory.  `stream` is a hipStream_t (NULL = the default stream); device work
 * is ordered on it and the call returns after the results it documents as
 * host outputs are written.  Handles are owned by the caller, who destroys
 * them; a handle is not used from two threads at once.
 */
#ifndef DLOOPS_H
#define DLOOPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DL_OK = 0,
    DL_EINVAL = -1,        /* invalid argument (nothing was done) */
    DL_ENOMEM = -2,        /* device allocation failed */
    DL_EHIP = -3,          /* a HIP runtime call failed */
    DL_ENOCONV = -4,       /* a solve did not reach its tolerance; best iterates written */
    DL_EBREAKDOWN = -5,    /* Krylov breakdown that a restart could not cure */
    DL_ENAN = -6,          /* non-finite value met in a solve */
    DL_EUNSUPPORTED = -7   /* valid but not supported combination */
} dl_status;

/* storage precision of fields and links; arithmetic is FP64 for DL_F64 and
   FP32 for the others (FP16 spinors carry one FP32 scale per site) */
typedef enum { DL_F64 = 0, DL_F32 = 1, DL_F16 = 2, DL_BF16 = 3 } dl_prec;

/* operators for dl_apply */
typedef enum {
    DL_OP_DHOP = 0,     /* D (hopping term), full lattice */
    DL_OP_M = 1,        /* M = 1 - kappa D */
    DL_OP_MDAG = 2,     /* M^dagger = 1 - kappa D^dagger */
    DL_OP_MHAT = 3,     /* even-site Schur complement 1 - kappa^2 D_eo D_oe (odd part of
                           input ignored, odd part of output set to zero) */
    DL_OP_MHATDAG = 4,  /* its adjoint */
    DL_OP_DHOPDAG = 5   /* D^dagger */
} dl_op;

typedef enum { DL_BICGSTAB = 0, DL_CGNR = 1 } dl_solver;

typedef enum { DL_SRC_Z2 = 0, DL_SRC_POINT = 1 } dl_source_kind;

typedef enum {
    DL_DIL_SPIN_COLOUR = 1,
    DL_DIL_CUBIC = 2,
    DL_DIL_EVEN_ODD = 4,
    DL_DIL_COLOUR = 8,
    DL_DIL_SPIN = 16,
    DL_DIL_SPIN_EVEN_ODD = 32,
    DL_DIL_TIME = 64
} dl_dilution_bits;

typedef struct dl_lattice_s *dl_lattice;
typedef struct dl_gauge_s *dl_gauge;

/* Description of the last failure on this thread ("" if none). */
const char *dl_last_error(void);

/* Library version string. */
const char *dl_version(void);

/*
 * Create a lattice description.  dims: host int32[4] = {X, Y, Z, T}, each even
 * and >= 2, V = XYZT <= 2^31 - 1.  t_antiperiodic: 1 = antiperiodic time
 * boundary (b = -1 on hops across it), 0 = periodic.  Space is periodic.
 * Errors: DL_EINVAL for a null pointer, odd or non-positive extents.
 */
int dl_lattice_create(const int32_t dims[4], int32_t t_antiperiodic, dl_lattice *out);
void dl_lattice_destroy(dl_lattice lat);

/* Lattice volume V (0 for a null handle). */
int64_t dl_lattice_volume(dl_lattice lat);

/*
 * Upload a gauge field: the SU(3) link variables U_mu(x) of the N_f = 2
 * Wilson-Dirac operator the paper inverts (Section 2: Wilson fermions on a
 * 16^3 x 32 ensemble; here any even lattice).  links: host canonical
 * complex128 [4][V][3][3] of special-unitary matrices (the third row is
 * rebuilt from the first two when recon = 12).  prec_mask: bit (1 << p) for
 * each dl_prec p to keep resident on the device.  recon: 12 (store two rows,
 * rebuild the third as the conjugated cross product) or 18 (store all three;
 * the only exact choice for links that are not special-unitary, e.g. when
 * differentiating with respect to unconstrained matrices).  The
 * time-boundary sign is never folded into the stored links (a negated
 * 12-parameter link would rebuild the wrong third row).  The handle keeps its
 * own copy of the lattice description; the lattice handle may be destroyed
 * after.  The caller's buffer is not referenced after the call returns.
 * Errors: DL_EINVAL (null pointers, empty mask, recon not 12 or 18),
 * DL_ENOMEM, DL_EHIP.
 */
int dl_gauge_create(dl_lattice lat, const double *links, uint32_t prec_mask, int32_t recon, void *stream,
                    dl_gauge *out);

/*
 * As dl_gauge_create, with the links in device memory (canonical complex128
 * [4][V][3][3], e.g. a torch tensor's data_ptr()): the reordering into the
 * library's layout runs on the device, ordered on `stream`; no host copy of
 * the field is made.  The caller's buffer is not referenced after the call
 * returns.  Errors as dl_gauge_create.
 */
int dl_gauge_create_device(dl_lattice lat, const void *links, uint32_t prec_mask, int32_t recon, void *stream,
                           dl_gauge *out);
void dl_gauge_destroy(dl_gauge g);

/*
 * out = op(in) for nrhs fields: the Wilson-Dirac matrix M = 1 - kappa D_hop
 * whose inverse the method needs (Section 2), its adjoint, the hopping term
 * alone, or the even-site Schur complement the even-odd preconditioned
 * solver iterates on (M = [[1, -k D_eo], [-k D_oe, 1]] in even-odd blocks,
 * so M^-1 restricted to even sites is the inverse of 1 - k^2 D_eo D_oe).
 * in, out: device canonical complex128 [nrhs][V][4][3], owned by the
 * caller; they must not overlap.  prec: storage precision of the links and
 * fields the operator runs in (must be resident in the gauge handle; the
 * reduced precisions of the truncated solver method, Section 2); results are
 * converted back to complex128.  kappa is ignored for DL_OP_DHOP /
 * DL_OP_DHOPDAG.  nrhs in [1, 65535].  Errors: DL_EINVAL (null pointer, nrhs
 * outside its range, unknown op, precision not resident, in == out),
 * DL_ENOMEM, DL_EHIP; out is undefined after an error other than DL_EINVAL.
 */
int dl_apply(dl_gauge g, double kappa, int32_t op, int32_t prec, const void *in, void *out, int64_t nrhs,
             void *stream);

/*
 * dl_apply for callers that cannot allocate device memory: code being
 * captured into a graph, tight serving loops, harnesses that forbid hipMalloc.
 * out = op(in) exactly as dl_apply (same arguments, layouts and errors), with
 * the packed parity fields in a static device scratch array of
 * DL_NOALLOC_SCRATCH_BYTES (64 MiB) instead of allocated workspaces; each GPU
 * the library runs on holds its own array until the process ends.  The call
 * needs 4 packed half fields (5 for DL_OP_MHAT / DL_OP_MHATDAG) of nrhs
 * right-hand sides in the storage precision, each rounded up to 256 bytes: at
 * 16^3 x 32 that is one right-hand side in FP64 or four in FP16.  A larger
 * request returns DL_EINVAL before any device work.  It calls no hipMalloc,
 * hipFree or other allocating routine: the launch configuration is the
 * autotuner's choice already in memory or its default (no tuning runs), and
 * no profiling events are recorded.  Unlike dl_apply the call does not
 * synchronise: out is complete when `stream` reaches the end of the call's
 * work.  Every call on one GPU shares that GPU's scratch and finds the last
 * call's contents there (every field is written before it is read): calls
 * ordered on one stream are safe, calls that overlap in time on one GPU
 * (other streams or threads) race.
 */
#define DL_NOALLOC_SCRATCH_BYTES 67108864
int dl_apply_noalloc(dl_gauge g, double kappa, int32_t op, int32_t prec, const void *in, void *out, int64_t nrhs,
                     void *stream);

/* Solver parameters. */
typedef struct {
    int32_t solver;      /* DL_BICGSTAB or DL_CGNR (CG on the normal equations of the Schur system) */
    int32_t prec;        /* storage precision of the iterated vectors; below DL_F64 a tolerance-driven
                            BiCGStab runs with FP64 reliable updates of x and of the residual */
    double tol;          /* stop when the FP64 true residual |b - M x| / |b| <= tol (fixed_iters = 0) */
    int32_t maxiter;     /* iteration cap (tolerance-driven solves) */
    int32_t fixed_iters; /* > 0: run exactly this many iterations from x0 = 0 (truncated solve) */
    double delta;        /* reliable-update trigger: |r| < delta * max |r| since the last update
                            (0 -> 0.01) */
    int32_t poll;        /* iterations between host convergence checks (0 -> automatic) */
    int32_t use_graph;   /* 1: capture `poll` BiCGStab iterations once as a hipGraph and replay it
                            (the first chunk runs eagerly and tunes the launch shapes).  A failure
                            during the capture ends it before the call returns, so the stream is
                            usable again.  For tests of that path, the environment variable
                            DL_FAULT_INJECT=capture makes every capture fail after it has begun. */
} dl_solve_params;

/* Per right-hand side results of a solve. */
typedef struct {
    int32_t status;           /* DL_OK, DL_ENOCONV, DL_ENAN */
    int32_t iters;            /* Krylov iterations */
    int32_t reliable_updates; /* FP64 residual replacements */
    int32_t pad;
    double true_rel_residual; /* FP64 |b - M x| / |b| of the returned solution (0 where not computed) */
    double seconds;           /* this right-hand side's share of the wall time of its batch (the
                                 batch's time divided by its right-hand sides) */
    double bytes;             /* algorithmic bytes of its field operands: every operand of every kernel
                                 its solve ran, moved once (per iteration 25 half fields for BiCGStab,
                                 19 for CGNR, in the iteration precision; per reliable update 8 FP64
                                 and 3 iteration-precision half fields; set-up and reconstruction); the
                                 links, shared by the batch, are not counted */
} dl_solve_stats;

/*
 * Solve M x = b for nrhs right-hand sides: the inversions the method consists
 * of (Section 2; the paper uses mixed-precision CG/BiCGStab, here even-odd
 * preconditioned BiCGStab with FP64 reliable updates, or the truncated CGNR
 * of the truncated solver method's low-precision solves).  Even-odd: the
 * Schur system (1 - k^2 D_eo D_oe) x_e = b_e + k D_eo b_o on even sites, then
 * x_o = b_o + k D_oe x_e.  A tolerance-driven solve has converged when the
 * FP64 true residual |b - M x| / |b| of the full system is <= tol.  b, x:
 * device canonical complex128 [nrhs][V][4][3], owned by the caller, not
 * overlapping.  stats: host [nrhs] or NULL.  Right-hand sides run in batches
 * that fit the workspace limit (DL_WORKSPACE_GB, default 160).  Returns
 * DL_ENOCONV if any tolerance-driven solve did not converge within maxiter
 * (x holds the last iterate, stats say which), DL_ENAN for a non-finite
 * value, DL_EINVAL for invalid arguments (before any device work).
 */
int dl_solve(dl_gauge g, double kappa, const dl_solve_params *params, const void *b, void *x, int64_t nrhs,
             dl_solve_stats *stats, void *stream);

/* Sources of a loop estimate. */
typedef struct {
    int32_t kind;        /* DL_SRC_Z2: complex Z2 noise; DL_SRC_POINT: the 12 unit sources at one site */
    int32_t scheme;      /* DL_SRC_Z2: dilution bits (0 = undiluted) */
    uint64_t seed;       /* DL_SRC_Z2: SplitMix64 seed */
    int64_t first_noise; /* DL_SRC_Z2: noise numbers first_noise .. first_noise + n_noise - 1 */
    int32_t n_noise;     /* DL_SRC_Z2: number of noise vectors; DL_SRC_POINT: must be 1 */
    int32_t point_site;  /* DL_SRC_POINT: lexicographic site index */
} dl_sources;

/*
 * Loop estimate (Sections 2-3): for every noise n and dilution class d solve
 * M s = eta_{n,d} and accumulate
 *     loops[n][g][t] = sum_d sum_{x: x_4 = t} eta_{n,d}(x)^+ Gamma_{gammas[g]} s(x),
 * a per-noise sum over dilution classes (not a mean).  For DL_SRC_POINT the
 * single "noise" is the set of 12 unit sources at point_site and
 * loops[0][g][t(site)] = Tr[Gamma M^-1(site, site)] exactly.
 * gammas: host int32[n_gamma], each in [0, 15], 1 <= n_gamma <= 16.
 * loops: host double [n_noise][n_gamma][T][2].  stats: host [n_noise * classes]
 * (right-hand side order: noise-major, then dilution class) or NULL.
 */
int dl_loops(dl_gauge g, double kappa, const dl_sources *src, const dl_solve_params *params,
             const int32_t *gammas, int32_t n_gamma, double *loops, dl_solve_stats *stats, void *stream);

/* Truncated solver method split (Section 2). */
typedef struct {
    int32_t n_lp;        /* noises first_noise .. first_noise + n_lp - 1: low-precision set */
    int32_t n_hp;        /* the next n_hp noises: high-precision correction set */
    dl_solve_params lp;  /* the truncated low-precision solve (e.g. DL_CGNR, DL_F16, fixed_iters 25) */
    dl_solve_params hp;  /* the high-precision solve (e.g. DL_BICGSTAB, DL_F32 with FP64 reliable updates, 1e-10) */
} dl_tsm;

/*
 * The truncated solver method's estimate and its variance (Section 2), in
 * FP64 on the host:
 *     est[g][t] = mean_{j in LP set} L^LP_j + mean_{j in HP set} (L^HP_j - L^LP_j),
 *     var[g][t] = s2(L^LP)/n_lp + s2(L^HP - L^LP)/n_hp,
 * s2 the unbiased sample variance of complex values (sum of |z - mean|^2 over
 * n - 1), i.e. the variance of est when the noises are independent.
 * lp_set_lp: host [n_lp][n_gamma][T][2] (the LP set's low-precision loops);
 * hp_set_hp, hp_set_lp: host [n_hp][n_gamma][T][2] (the HP set's high- and
 * low-precision loops) -- the three blocks of the dl_loops_tsm output, or any
 * resampling of them.  est: host [n_gamma][T][2]; var: host [n_gamma][T] or
 * NULL.  Errors: DL_EINVAL (null pointer, n_lp or n_hp < 1, or < 2 when var
 * is requested, n_gamma outside [1, 16], T outside [1, 65535]).
 */
int dl_tsm_combine(const double *lp_set_lp, int32_t n_lp, const double *hp_set_hp, const double *hp_set_lp,
                   int32_t n_hp, int32_t n_gamma, int32_t T, double *est, double *var);

/*
 * Truncated solver method (Section 2): low-precision solves on all
 * n_lp + n_hp noises of src (src->n_noise must equal n_lp + n_hp) and
 * high-precision solves on the n_hp correction noises.  loops: host double
 * [n_lp + 2 n_hp][n_gamma][T][2] holding, per noise as in dl_loops, first the
 * LP-set low-precision loops, then the HP-set high-precision loops, then the
 * HP-set low-precision loops.  The estimate is mean(LP set, low) +
 * mean(HP set, high - low), formed with its variance by dl_tsm_combine.
 * stats: host [(n_lp + n_hp) * classes + n_hp * classes] (the
 * low-precision solves, then the high-precision ones) or NULL.
 */
int dl_loops_tsm(dl_gauge g, double kappa, const dl_sources *src, const dl_tsm *tsm, const int32_t *gammas,
                 int32_t n_gamma, double *loops, dl_solve_stats *stats, void *stream);

/*
 * Derivative of the loop estimator with respect to kappa: since
 * dM^-1/dkappa = M^-1 D M^-1, dloops[n][g][t] = sum_d eta_d^+ P_t Gamma u_d with
 * u_d = M^-1 D M^-1 eta_d (two solves per right-hand side, tolerance-driven
 * BiCGStab only).  dloops: host double [n_noise][n_gamma][T][2].  stats: host
 * [2][n_noise * classes] (first and second solves) or NULL.
 */
int dl_loops_dkappa(dl_gauge g, double kappa, const dl_sources *src, const dl_solve_params *params,
                    const int32_t *gammas, int32_t n_gamma, double *dloops, dl_solve_stats *stats, void *stream);

/*
 * Gradient of the real functional F = Re sum_{n,g,t} conj(w[n][g][t]) loops[n][g][t]
 * with respect to the gauge links, each U_mu(x) taken as an unconstrained 3x3
 * complex matrix: grad[mu][x][a][b] = dF/dRe U_ab + i dF/dIm U_ab (so
 * dF = Re sum conj(grad) dU).  With s = M^-1 eta and the adjoint solution
 * a = M^-dagger (sum_g w Gamma_g^+ P_t eta) = gamma5 M^-1 gamma5 (...), the
 * variation is dF = Re kappa sum a^+ dD s (two solves per right-hand side,
 * tolerance-driven BiCGStab only).  w: host double [n_noise][n_gamma][T][2]
 * (the cotangent of the loops).  grad: host or device double
 * [4][V][3][3][2] (overwritten).  loops: host [n_noise][n_gamma][T][2] or
 * NULL (the forward loops, as dl_loops).  dloops: host
 * [n_noise][n_gamma][T][2] or NULL (the kappa derivative, as
 * dl_loops_dkappa, at the cost of a third solve).  dF_dkappa: host double or
 * NULL: dF/dkappa = Re sum conj(w) dloops (also a third solve).  stats: host
 * [2 or 3][n_noise * classes] (forward, adjoint, kappa solves) or NULL.
 */
int dl_loops_link_grad(dl_gauge g, double kappa, const dl_sources *src, const dl_solve_params *params,
                       const int32_t *gammas, int32_t n_gamma, const double *w, double *grad, double *loops,
                       double *dloops, double *dF_dkappa, dl_solve_stats *stats, void *stream);

/*
 * Loop estimates on up to 4 lattices of different shapes at once (each with
 * its own gauge field, kappa and sources; one solver parameter set): every
 * solver step is one launch over all lattices' right-hand sides, with
 * params->use_graph replaying the captured iteration chunks.  Results per
 * lattice exactly as dl_loops: loops[l] host [n_noise_l][n_gamma][T_l][2],
 * stats[l] host [n_noise_l * classes_l] (stats or stats[l] may be NULL).
 * Tolerance-driven BiCGStab only.  Errors: DL_EINVAL (n_lat outside [1, 4],
 * null pointers, invalid sources or parameters).
 */
int dl_batch_loops(int32_t n_lat, const dl_gauge *gauges, const double *kappas, const dl_sources *srcs,
                   const dl_solve_params *params, const int32_t *gammas, int32_t n_gamma, double *const *loops,
                   dl_solve_stats *const *stats, void *stream);

/* Number of right-hand sides (solves) a dl_sources description expands to, or < 0 if invalid. */
int64_t dl_sources_count(dl_lattice lat, const dl_sources *src);

/*
 * Write right-hand sides first_rhs .. first_rhs + nrhs - 1 of a dl_sources
 * description (noise-major, then dilution class) into out: device canonical
 * complex128 [nrhs][V][4][3].  These are exactly the vectors dl_loops solves
 * for.  Errors: DL_EINVAL (invalid sources, range outside [0, count)).
 */
int dl_sources_fill(dl_lattice lat, const dl_sources *src, int64_t first_rhs, int64_t nrhs, void *out, void *stream);

/*
 * Gauge-covariant Gaussian smearing of quark fields (Section 2; the paper
 * uses it for smeared meson operators and gives no parameters):
 *     S = F^iters,  (F psi)(x) = [ psi(x) + alpha sum_{i=x,y,z} ( U_i(x) psi(x+i)
 *                                  + U_i(x-i)^+ psi(x-i) ) ] / (1 + 6 alpha),
 * spin-diagonal, within each timeslice, periodic in space; S is hermitian.
 * dl_smear: out = S in for device canonical complex128 [nrhs][V][4][3]
 * fields (in and out must not overlap), computed in FP64 with the FP64 links.
 * alpha finite and >= 0, iters in [0, 100000] (0 copies), nrhs in
 * [1, 65535]; the gauge handle must hold FP64 links; else DL_EINVAL.
 */
int dl_smear(dl_gauge g, double alpha, int32_t iters, const void *in, void *out, int64_t nrhs, void *stream);

/*
 * Loops of smeared quark fields: as dl_loops, with the local loop of the
 * smeared propagator S M^-1 S,
 *     loops[n][g][t] = sum_d sum_{x: x_4 = t} xi_{n,d}(x)^+ Gamma s(x),
 *     xi_{n,d} = S eta_{n,d},  M s = xi_{n,d},
 * (S acts within timeslices and not on spin, and is hermitian, so smearing
 * the sink is the same as contracting with the smeared noise).  Smearing runs
 * in FP64; the solve as params says.  Arguments as dl_loops plus alpha and
 * iters as dl_smear.
 */
int dl_loops_smeared(dl_gauge g, double kappa, const dl_sources *sources, double alpha, int32_t iters,
                     const dl_solve_params *params, const int32_t *gammas, int32_t n_gamma, double *loops,
                     dl_solve_stats *stats, void *stream);

/*
 * Disconnected two-loop correlator at zero momentum (Section 3, Eq. 2) from
 * per-noise loop estimates of two insertions B and A, e.g. two Gamma slices
 * of the dl_loops output (one lattice, one set of noises):
 *     corr[dt] = -1/(spatial_volume * T) * 1/(n (n - 1))
 *                * sum_{n' != m} sum_t L_B^{n'}(t) L_A^{m}((t + dt) mod T),
 * i.e. the noise expectation of the product of two loops is estimated over
 * ordered pairs of distinct noises: the product of two estimates on the same
 * noise carries that noise's own fluctuation as a bias.  (The expectation
 * over gauge fields is the caller's.)
 * loops_b, loops_a: host [n_noise][T][2] (re, im) FP64; corr: host [T][2],
 * indexed by dt = 0 .. T-1.  Summation order is fixed (run-to-run
 * deterministic).  n_noise >= 2, T in [1, 65535], spatial_volume >= 1 and
 * non-null pointers, else DL_EINVAL before any device work.  Runs on `stream`
 * (null = default) and returns after the result has been copied back.
 */
int dl_disconnected_correlator(const double *loops_b, const double *loops_a, int32_t n_noise, int32_t T,
                               int64_t spatial_volume, double *corr, void *stream);

/*
 * The flavour-singlet pseudoscalar combination and the ratio fit of Section 3
 * (Eqs. 3 and 4), on correlators the caller has averaged per gauge
 * configuration: d[n][t] the disconnected correlator D(t) (e.g. the real part
 * of dl_disconnected_correlator), c_pi[n][t] the connected pion correlator
 * C_pi(t), n = 0 .. ncfg-1, t = 0 .. T-1 (host, row-major FP64).
 *     c_eta[t] = mean_n (C_pi - 2 D)(t)                            (Eq. 3)
 *     R(t) = sum_n D / sum_n C_pi  fitted on tmin <= t <= tmax to
 *     A - B (e^{-m t} + e^{-m (T - t)}) / (e^{-m_pi t} + e^{-m_pi (T - t)})   (Eq. 4)
 * with m_pi given (the prior): params[3] = (A, B, m) where m is the
 * eta' mass, the one minimising chi^2 = sum_t w_t (R - model)^2 over m in
 * [1e-3, 10] (lattice units); w_t = 1 / var R(t) from a jackknife over
 * configurations when ncfg >= 2 (unit weights otherwise, or where a variance
 * vanishes).  errors[3]: jackknife errors of (A, B, m) (each sample refitted
 * with the same weights; zeros when ncfg < 2).  *chi2: the fit's chi^2.
 * Host computation, no device work.  Returns DL_EINVAL for a null pointer,
 * ncfg < 1, T outside [4, 65535], fewer than 4 points in [tmin, tmax] (or
 * the range outside [0, T)), m_pi <= 0, or a zero / non-finite configuration
 * sum of C_pi in the fit range.
 */
int dl_eta_prime_fit(const double *d, const double *c_pi, int32_t ncfg, int32_t T, double m_pi, int32_t tmin,
                     int32_t tmax, double *c_eta, double *params, double *errors, double *chi2);

/*
 * Device memory cache.  The library keeps the device buffers its calls
 * release (workspaces, staging) and serves later calls of the same shape from
 * them instead of allocating again; mapping multi-GB workspaces anew would
 * otherwise cost seconds per call.  A released buffer carries an event
 * recorded on the releasing call's stream, and a later call that takes it
 * waits for that event first.  The cached bytes are capped: the environment
 * variable DL_CACHE_GB (read at the first release; default 64, 0 disables
 * caching) or dl_cache_set_limit.  An allocation that fails releases the
 * cache and retries once.  Cached memory is not available to other
 * allocators (e.g. torch's) until it is released.
 * dl_cache_release frees every cached buffer (after waiting for its last
 * user) and returns DL_OK.  dl_cache_set_limit sets the cap in bytes (0 turns
 * caching off) and frees cached buffers beyond it.  dl_cache_bytes returns
 * the bytes held.
 */
int dl_cache_release(void);
int dl_cache_set_limit(uint64_t bytes);
uint64_t dl_cache_bytes(void);

/*
 * Kernel profiling on the library's streams.  dl_profile_enable(1) resets the
 * counters and brackets every following launch with HIP events (and a device
 * counter of the right-hand sides a hopping launch actually processed);
 * dl_profile_enable(0) stops.  Not for use while a stream is being captured.
 * dl_profile_read(kind, ms, bytes) synchronises and returns the number of
 * launches of that kind, their summed event-timed duration and their
 * algorithmic bytes (every operand moved once; for the hopping kernel, the
 * links once per launch plus the in/out/epilogue half spinors of each live
 * right-hand side).  kind: 0 = all hopping kernels, 1 = Krylov vector
 * kernels, 2 = sources and traces, 3 = the plain (no epilogue, not adjoint)
 * hopping kernel, 4 = smearing steps.  Returns DL_EINVAL for another kind.
 */
int dl_profile_enable(int32_t on);
int64_t dl_profile_read(int32_t kind, double *ms, double *bytes);

/*
 * Launch configuration of the most recent profiled hopping launch of profile
 * kind 0 (any hopping launch) or 3 (the plain one), as chosen by the
 * autotuner: cfg[0] = kernel (0 = item kernel, one thread per site and
 * cfg[1] right-hand sides; 1 = LDS-link kernel, links of a 64-site block in
 * LDS and cfg[1] wavefronts walking the right-hand sides), cfg[2] = sites per
 * workgroup (item kernel) or the wavefronts per SIMD the LDS-link kernel
 * allows (0 = as compiled), cfg[3] = persistent grid cap (item kernel, 0 =
 * none) or region size in site blocks (LDS-link kernel).  cfg (host, 4
 * int32) is all -1 when no such launch was profiled since
 * dl_profile_enable(1).  Returns DL_EINVAL for another kind or a null cfg.
 */
int dl_profile_config(int32_t kind, int32_t *cfg);

/*
 * Measurement helper, not part of the method: the rate the memory system
 * gives the library's own access pattern, to compare kernels with.  Mode 0
 * (copy) reads `bytes` of src and writes them to dst; mode 1 (read) reads
 * `bytes` of src and writes nothing but, should the running XOR of a thread's
 * words hit one fixed value, one 16-byte word per workgroup to dst (dst must
 * hold 128 KiB).  Both use 16-byte non-temporal loads (and stores): up to
 * 8192 workgroups of 256 threads walk tiles of 2048 contiguous words, eight
 * loads in flight per thread, each wavefront instruction covering 1 KiB, as
 * the field kernels access a component plane.  The pass runs `reps` times on
 * `stream` between HIP events and *seconds receives the mean time of one
 * pass.  src and dst are device pointers, 16-byte aligned and not
 * overlapping, bytes a non-zero multiple of 16; DL_EINVAL otherwise.
 */
int dl_stream_probe(const void *src, void *dst, uint64_t bytes, int32_t mode, int32_t reps, void *stream,
                    double *seconds);

#ifdef __cplusplus
}
#endif

#endif /* DLOOPS_H */

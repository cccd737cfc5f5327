/*
 * wilson_oracle.c -- plain, slow FP64 CPU oracle for the disconnected-loop
 * method of Alexandrou, Christaras, O Cais and Strelchenko, "Exact calculation
 * of disconnected loops" (Lattice 2010).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * Everything here is written straight from the definitions, in FP64, on the
 * full lattice (no even-odd splitting except where an algorithm's own steps
 * need it), with the 4x4 spin matrices applied as full matrices.
 *
 * Conventions (the paper names Wilson fermions and refers to a Dirac basis but writes
 * neither down; these are the readings used throughout):
 *   - site index  i = x + X*(y + Y*(z + Z*t)), direction mu = 0,1,2,3 = x,y,z,t;
 *   - spinor  psi[((i*4 + spin)*3 + colour)], complex;
 *   - links   U[((mu*V + i)*3 + a)*3 + b] = U_mu(x)_{ab}, complex;
 *   - chiral basis gamma_k = [[0,-i s_k],[i s_k,0]], gamma_4 = [[0,1],[1,0]],
 *     gamma_5 = g1 g2 g3 g4 = diag(1,1,-1,-1);
 *   - Wilson r = 1, hopping term (Section 2: N_f = 2 Wilson fermions)
 *       (D psi)(x) = sum_mu (1 - g_mu) b U_mu(x) psi(x+mu)
 *                         + (1 + g_mu) b U_mu(x-mu)^+ psi(x-mu),
 *     M = 1 - kappa D, b = -1 on the hop across the time boundary when the
 *     time direction is antiperiodic, +1 otherwise;
 *   - Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3, n = n0 + 2 n1 + 4 n2 + 8 n3.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* Geometry                                                            */
/* ------------------------------------------------------------------ */

static int64_t volume(const int32_t *L) { return (int64_t)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int32_t *L, int64_t i, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(i % L[mu]);
        i /= L[mu];
    }
}

static int64_t index_of(const int32_t *L, const int c[4])
{
    return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

/* neighbour of site i one step in direction mu, forward (dir=+1) or back (dir=-1) */
static int64_t hop(const int32_t *L, int64_t i, int mu, int dir)
{
    int c[4];
    coords(L, i, c);
    c[mu] = (c[mu] + dir + L[mu]) % L[mu];
    return index_of(L, c);
}

int32_t or_parity(const int32_t *L, int64_t i)
{
    int c[4];
    coords(L, i, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

int32_t or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Dirac algebra                                                       */
/* ------------------------------------------------------------------ */

static void mat4_mul(const cplx a[4][4], const cplx b[4][4], cplx out[4][4])
{
    cplx t[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
            t[i][j] = s;
        }
    memcpy(out, t, sizeof t);
}

/* gamma_{mu+1} for mu = 0..3 in the chiral basis */
static void gamma_mu(int mu, cplx g[4][4])
{
    const cplx J = _Complex_I;
    cplx sigma[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -J}, {J, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(g, 0, sizeof(cplx) * 16);
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            if (mu < 3) {
                g[r][c + 2] = -J * sigma[mu][r][c];
                g[r + 2][c] = J * sigma[mu][r][c];
            } else {
                g[r][c + 2] = (r == c) ? 1 : 0;
                g[r + 2][c] = (r == c) ? 1 : 0;
            }
        }
}

static void gamma_n(int n, cplx G[4][4])
{
    memset(G, 0, sizeof(cplx) * 16);
    for (int i = 0; i < 4; ++i) G[i][i] = 1;
    for (int mu = 0; mu < 4; ++mu)
        if ((n >> mu) & 1) {
            cplx g[4][4];
            gamma_mu(mu, g);
            mat4_mul(G, g, G);
        }
}

/* exported: Gamma_n as [4][4][re,im] */
void or_gamma(int32_t n, double *out)
{
    cplx G[4][4];
    gamma_n(n, G);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            out[2 * (4 * i + j)] = creal(G[i][j]);
            out[2 * (4 * i + j) + 1] = cimag(G[i][j]);
        }
}

/* ------------------------------------------------------------------ */
/* Hopping term D and its adjoint, written out from the definition     */
/* ------------------------------------------------------------------ */

/* boundary factor of the hop from site c in direction mu (dir = +-1) */
static double bc_sign(const int32_t *L, int tap, const int c[4], int mu, int dir)
{
    if (!tap || mu != 3) return 1.0;
    if (dir > 0 && c[3] == L[3] - 1) return -1.0;
    if (dir < 0 && c[3] == 0) return -1.0;
    return 1.0;
}

/*
 * out = D in          (dag = 0)
 * out = D^dagger in   (dag = 1), assembled directly as
 *   (D^+ psi)(x) = sum_mu (1 + g_mu) b U_mu(x) psi(x+mu) + (1 - g_mu) b U_mu(x-mu)^+ psi(x-mu)
 * i.e. the adjoint of every block of D, not via gamma_5.
 */
static void dhop_any(const int32_t *L, int tap, const cplx *U, const cplx *in, cplx *out, int dag)
{
    const int64_t V = volume(L);
    cplx gam[4][4][4];
    for (int mu = 0; mu < 4; ++mu) gamma_mu(mu, gam[mu]);

#pragma omp parallel for schedule(static) if (V >= 1024)
    for (int64_t i = 0; i < V; ++i) {
        int c[4];
        coords(L, i, c);
        cplx acc[4][3];
        memset(acc, 0, sizeof acc);
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = -1; dir <= 1; dir += 2) {
                /* spin matrix (1 - s g_mu): s = +1 forward, -1 backward for D;
                   flipped for D^dagger */
                double s = (dir > 0) ? 1.0 : -1.0;
                if (dag) s = -s;
                cplx P[4][4];
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) P[a][b] = (a == b ? 1.0 : 0.0) - s * gam[mu][a][b];
                const int64_t j = hop(L, i, mu, dir);
                const double b = bc_sign(L, tap, c, mu, dir);
                /* colour matrix: U_mu(x) forward, U_mu(x-mu)^dagger backward */
                cplx W[3][3];
                if (dir > 0) {
                    const cplx *u = U + (mu * V + i) * 9;
                    for (int a = 0; a < 3; ++a)
                        for (int bb = 0; bb < 3; ++bb) W[a][bb] = u[3 * a + bb];
                } else {
                    const cplx *u = U + (mu * V + j) * 9;
                    for (int a = 0; a < 3; ++a)
                        for (int bb = 0; bb < 3; ++bb) W[a][bb] = conj(u[3 * bb + a]);
                }
                const cplx *p = in + j * 12;
                for (int al = 0; al < 4; ++al)
                    for (int a = 0; a < 3; ++a) {
                        cplx sum = 0;
                        for (int be = 0; be < 4; ++be)
                            for (int bb = 0; bb < 3; ++bb) sum += P[al][be] * W[a][bb] * p[3 * be + bb];
                        acc[al][a] += b * sum;
                    }
            }
        }
        memcpy(out + i * 12, acc, sizeof acc);
    }
}

void or_dhop(const int32_t *L, int32_t tap, const double *U, const double *in, double *out)
{
    dhop_any(L, tap, (const cplx *)U, (const cplx *)in, (cplx *)out, 0);
}

void or_dhop_dag(const int32_t *L, int32_t tap, const double *U, const double *in, double *out)
{
    dhop_any(L, tap, (const cplx *)U, (const cplx *)in, (cplx *)out, 1);
}

/*
 * Gauge-covariant Gaussian smearing of quark fields (Section 2; the paper
 * names the method but gives no parameters), one step:
 *   (F psi)(x) = [ psi(x) + alpha sum_{i = x,y,z} ( U_i(x) psi(x+i) + U_i(x-i)^+ psi(x-i) ) ] / (1 + 6 alpha),
 * spin-diagonal, within each timeslice, periodic in space (no boundary sign).
 * out = F^iters in.
 */
void or_smear(const int32_t *L, const double *Ud, double alpha, int32_t iters, const double *in_d, double *out_d)
{
    const int64_t V = volume(L);
    const cplx *U = (const cplx *)Ud;
    cplx *a = malloc(sizeof(cplx) * V * 12), *b = malloc(sizeof(cplx) * V * 12);
    memcpy(a, in_d, sizeof(cplx) * V * 12);
    const double norm = 1.0 / (1.0 + 6.0 * alpha);
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static) if (V >= 1024)
        for (int64_t i = 0; i < V; ++i) {
            cplx acc[12];
            for (int k = 0; k < 12; ++k) acc[k] = 0;
            for (int mu = 0; mu < 3; ++mu)
                for (int dir = -1; dir <= 1; dir += 2) {
                    const int64_t j = hop(L, i, mu, dir);
                    cplx W[3][3];
                    if (dir > 0) {
                        const cplx *u = U + (mu * V + i) * 9;
                        for (int r = 0; r < 3; ++r)
                            for (int q = 0; q < 3; ++q) W[r][q] = u[3 * r + q];
                    } else {
                        const cplx *u = U + (mu * V + j) * 9;
                        for (int r = 0; r < 3; ++r)
                            for (int q = 0; q < 3; ++q) W[r][q] = conj(u[3 * q + r]);
                    }
                    const cplx *p = a + j * 12;
                    for (int sp = 0; sp < 4; ++sp)
                        for (int r = 0; r < 3; ++r)
                            for (int q = 0; q < 3; ++q) acc[3 * sp + r] += W[r][q] * p[3 * sp + q];
                }
            for (int k = 0; k < 12; ++k) b[i * 12 + k] = (a[i * 12 + k] + alpha * acc[k]) * norm;
        }
        cplx *t = a;
        a = b;
        b = t;
    }
    memcpy(out_d, a, sizeof(cplx) * V * 12);
    free(a);
    free(b);
}

/* out = M in = in - kappa D in  (dag selects M^dagger = 1 - kappa D^dagger) */
static void apply_m(const int32_t *L, int tap, const cplx *U, double kappa, const cplx *in, cplx *out,
                    int dag)
{
    const int64_t n = volume(L) * 12;
    cplx *t = malloc(sizeof(cplx) * n);
    dhop_any(L, tap, U, in, t, dag);
#pragma omp parallel for schedule(static) if (n >= 65536)
    for (int64_t k = 0; k < n; ++k) out[k] = in[k] - kappa * t[k];
    free(t);
}

void or_apply_m(const int32_t *L, int32_t tap, const double *U, double kappa, const double *in, double *out)
{
    apply_m(L, tap, (const cplx *)U, kappa, (const cplx *)in, (cplx *)out, 0);
}

void or_apply_mdag(const int32_t *L, int32_t tap, const double *U, double kappa, const double *in,
                   double *out)
{
    apply_m(L, tap, (const cplx *)U, kappa, (const cplx *)in, (cplx *)out, 1);
}

/* ------------------------------------------------------------------ */
/* Vector helpers                                                      */
/* ------------------------------------------------------------------ */

static cplx dot(const cplx *a, const cplx *b, int64_t n)
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static) if (n >= 65536)
    for (int64_t k = 0; k < n; ++k) {
        cplx z = conj(a[k]) * b[k];
        re += creal(z);
        im += cimag(z);
    }
    return re + _Complex_I * im;
}

static double norm2(const cplx *a, int64_t n) { return creal(dot(a, a, n)); }

/* ------------------------------------------------------------------ */
/* BiCGStab on the full lattice, M x = b, x0 = 0                       */
/* ------------------------------------------------------------------ */

/*
 * Textbook BiCGStab (van der Vorst 1992) on the unpreconditioned full-lattice
 * matrix.  The stopping test is the true residual |b - M x| / |b| <= tol,
 * recomputed in FP64; when the iterated residual says "converged" but the
 * true one does not (or on a breakdown), the iteration restarts from the true
 * residual.  Returns the number of iterations used, or -1 if tol was not met.
 * *true_res receives the final true relative residual.
 */
int32_t or_bicgstab(const int32_t *L, int32_t tap, const double *Ud, double kappa, const double *bd,
                    double *xd, double tol, int32_t maxiter, double *true_res)
{
    const cplx *U = (const cplx *)Ud, *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    const int64_t n = volume(L) * 12;
    cplx *r = malloc(sizeof(cplx) * n), *rh = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n),
         *v = malloc(sizeof(cplx) * n), *s = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    const double bnorm = sqrt(norm2(b, n));
    memset(x, 0, sizeof(cplx) * n);
    int it = 0, restarts = 0;
    double res = 0, best = INFINITY;
    if (bnorm == 0) {
        *true_res = 0;
        free(r); free(rh); free(p); free(v); free(s); free(t);
        return 0;
    }
    for (;;) {
        /* (re)start from the true residual */
        apply_m(L, tap, U, kappa, x, t, 0);
        for (int64_t k = 0; k < n; ++k) r[k] = b[k] - t[k];
        res = sqrt(norm2(r, n)) / bnorm;
        /* stop when converged, out of iterations, or when a restart no longer
           improves the true residual (rounding floor reached) */
        if (res <= tol || it >= maxiter || (restarts > 0 && res >= 0.5 * best)) break;
        if (res < best) best = res;
        ++restarts;
        memcpy(rh, r, sizeof(cplx) * n);
        memset(p, 0, sizeof(cplx) * n);
        memset(v, 0, sizeof(cplx) * n);
        cplx rho = 1, alpha = 1, omega = 1;
        while (it < maxiter) {
            cplx rho_new = dot(rh, r, n);
            if (rho_new == 0) break; /* breakdown: restart from the true residual */
            cplx beta = (rho_new / rho) * (alpha / omega);
            for (int64_t k = 0; k < n; ++k) p[k] = r[k] + beta * (p[k] - omega * v[k]);
            apply_m(L, tap, U, kappa, p, v, 0);
            alpha = rho_new / dot(rh, v, n);
            for (int64_t k = 0; k < n; ++k) s[k] = r[k] - alpha * v[k];
            ++it;
            if (sqrt(norm2(s, n)) / bnorm <= tol) {
                for (int64_t k = 0; k < n; ++k) x[k] += alpha * p[k];
                break;
            }
            apply_m(L, tap, U, kappa, s, t, 0);
            double tt = norm2(t, n);
            omega = tt > 0 ? dot(t, s, n) / tt : 0;
            for (int64_t k = 0; k < n; ++k) {
                x[k] += alpha * p[k] + omega * s[k];
                r[k] = s[k] - omega * t[k];
            }
            rho = rho_new;
            if (omega == 0) break;
            if (sqrt(norm2(r, n)) / bnorm <= tol) break;
        }
    }
    *true_res = res;
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return res <= tol ? it : -1;
}

/* ------------------------------------------------------------------ */
/* Even-odd pieces, used only where an algorithm's own steps need them */
/* ------------------------------------------------------------------ */

/* zero every entry on sites of the given parity */
static void zero_parity(const int32_t *L, cplx *v, int parity)
{
    const int64_t V = volume(L);
    for (int64_t i = 0; i < V; ++i)
        if (or_parity(L, i) == parity)
            for (int k = 0; k < 12; ++k) v[i * 12 + k] = 0;
}

/*
 * Schur complement on even sites: with M = [[1, -k D_eo], [-k D_oe, 1]],
 *   Mhat x_e = x_e - k^2 D_eo D_oe x_e.
 * For a vector supported on even sites, D maps it to odd sites and D again
 * back to even sites, so Mhat x = x - k^2 D(D x).  dag = 1 gives
 * Mhat^dagger = 1 - k^2 (D^dagger)_eo (D^dagger)_oe.
 */
static void apply_mhat(const int32_t *L, int tap, const cplx *U, double kappa, const cplx *in, cplx *out,
                       int dag)
{
    const int64_t n = volume(L) * 12;
    cplx *t = malloc(sizeof(cplx) * n), *u = malloc(sizeof(cplx) * n);
    dhop_any(L, tap, U, in, t, dag);
    dhop_any(L, tap, U, t, u, dag);
    for (int64_t k = 0; k < n; ++k) out[k] = in[k] - kappa * kappa * u[k];
    free(t);
    free(u);
}

void or_apply_mhat(const int32_t *L, int32_t tap, const double *U, double kappa, const double *in,
                   double *out, int32_t dag)
{
    apply_mhat(L, tap, (const cplx *)U, kappa, (const cplx *)in, (cplx *)out, dag);
}

/*
 * The low-precision solve of the truncated solver method, run here in FP64:
 * conjugate gradient on the normal equations of the even-site Schur system,
 *   Mhat^+ Mhat x_e = Mhat^+ bhat_e,  bhat_e = b_e + k D_eo b_o,  x0 = 0,
 * stopped after exactly niter iterations, followed by x_o = b_o + k D_oe x_e.
 * With niter = 0 it returns x_e = 0, x_o = b_o.
 */
void or_cgnr_eo(const int32_t *L, int32_t tap, const double *Ud, double kappa, const double *bd, double *xd,
                int32_t niter)
{
    const cplx *U = (const cplx *)Ud, *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    const int64_t n = volume(L) * 12;
    cplx *bo = malloc(sizeof(cplx) * n), *bh = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n),
         *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    /* bhat_e = b_e + k D b_o restricted to even sites */
    memcpy(bo, b, sizeof(cplx) * n);
    zero_parity(L, bo, 0);
    dhop_any(L, tap, U, bo, t, 0);
    for (int64_t k = 0; k < n; ++k) bh[k] = b[k] + kappa * t[k];
    zero_parity(L, bh, 1);
    /* r = Mhat^+ bhat, x = 0 */
    apply_mhat(L, tap, U, kappa, bh, r, 1);
    memset(x, 0, sizeof(cplx) * n);
    memcpy(p, r, sizeof(cplx) * n);
    double rr = norm2(r, n);
    for (int it = 0; it < niter && rr > 0; ++it) {
        apply_mhat(L, tap, U, kappa, p, t, 0);
        apply_mhat(L, tap, U, kappa, t, q, 1);
        double pq = creal(dot(p, q, n));
        if (!(pq > 0)) break; /* exact convergence: nothing left to do */
        double alpha = rr / pq;
        for (int64_t k = 0; k < n; ++k) {
            x[k] += alpha * p[k];
            r[k] -= alpha * q[k];
        }
        double rr_new = norm2(r, n);
        double beta = rr_new / rr;
        for (int64_t k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
        rr = rr_new;
    }
    /* x_o = b_o + k D x_e */
    dhop_any(L, tap, U, x, t, 0);
    for (int64_t i = 0; i < volume(L); ++i)
        if (or_parity(L, i) == 1)
            for (int k = 0; k < 12; ++k) x[i * 12 + k] = b[i * 12 + k] + kappa * t[i * 12 + k];
    free(bo); free(bh); free(t); free(r); free(p); free(q);
}

/* ------------------------------------------------------------------ */
/* Noise: complex Z2 from SplitMix64 (Steele, Lea and Flood, 2014)     */
/* ------------------------------------------------------------------ */

/*
 * Output number c (0-based) of the SplitMix64 stream seeded with `seed`.
 * The generator's state advances by the golden-ratio increment before each
 * output, so the state behind output c is seed + (c+1)*increment (mod 2^64);
 * the output is that state pushed through the published 64-bit finaliser.
 */
uint64_t or_splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/*
 * Complex Z2 noise entry (+-1 +-i)/sqrt(2) for (noise, site, spin, colour):
 * counter c = ((noise*V + site)*4 + spin)*3 + colour; bit 0 of the draw sets
 * the sign of the real part, bit 1 that of the imaginary part (0 -> +).
 */
static cplx z2_entry(uint64_t seed, int64_t V, int64_t noise, int64_t site, int spin, int col)
{
    uint64_t c = (uint64_t)(((noise * V + site) * 4 + spin) * 3 + col);
    uint64_t r = or_splitmix64(seed, c);
    double re = (r & 1) ? -1.0 : 1.0, im = (r & 2) ? -1.0 : 1.0;
    /* sqrt(0.5) is the correctly rounded 1/sqrt(2) (one rounding, not two) */
    return (re + _Complex_I * im) * sqrt(0.5);
}

/*
 * Dilution class of entry (site, spin, colour) under a scheme (Section 2):
 *   scheme bit 0 (1): spin-colour dilution, class 3*spin + colour (12);
 *   scheme bit 4 (16): spin dilution, class spin (4);
 *   scheme bit 5 (32): spin even-odd partitioning, class spin & 1 (2);
 *   scheme bit 3 (8): colour dilution, class colour (3);
 *   scheme bit 1 (2): cubic spatial dilution, class (x&1) + 2(y&1) + 4(z&1) (8);
 *   scheme bit 2 (4): spatial even-odd dilution, class (x+y+z+t)&1 (2).
 * Classes of the enabled factors combine in the order listed, each later
 * factor being the faster-running digit, so spin + colour (16 | 8) gives the
 * same classes as spin-colour (1).  Bit 0 excludes bits 3-5; bits 4 and 5
 * exclude each other (or_dilution_valid).
 *   scheme bit 6 (64): time dilution, one class: noise n is supported on
 * timeslice n mod T only (or_z2_source), so every noise costs the same
 * number of solves and the timeslices are covered across noises.
 */
int32_t or_dilution_valid(int32_t scheme)
{
    if (scheme < 0 || scheme > 127) return 0;
    if ((scheme & 1) && (scheme & (8 | 16 | 32))) return 0;
    if ((scheme & 16) && (scheme & 32)) return 0;
    return 1;
}

int32_t or_dilution_class(const int32_t *L, int32_t scheme, int64_t site, int32_t spin, int32_t col)
{
    int c[4];
    coords(L, site, c);
    int32_t d = 0;
    if (scheme & 1) d = d * 12 + 3 * spin + col;
    if (scheme & 16) d = d * 4 + spin;
    if (scheme & 32) d = d * 2 + (spin & 1);
    if (scheme & 8) d = d * 3 + col;
    if (scheme & 2) d = d * 8 + (c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1);
    if (scheme & 4) d = d * 2 + ((c[0] + c[1] + c[2] + c[3]) & 1);
    return d;
}

int32_t or_dilution_count(int32_t scheme)
{
    return ((scheme & 1) ? 12 : 1) * ((scheme & 16) ? 4 : 1) * ((scheme & 32) ? 2 : 1) * ((scheme & 8) ? 3 : 1) *
           ((scheme & 2) ? 8 : 1) * ((scheme & 4) ? 2 : 1);
}

/* eta_{noise,d}: the noise vector masked to dilution class d (d = -1: no class
 * mask); under time dilution also masked to timeslice noise mod T */
void or_z2_source(const int32_t *L, uint64_t seed, int64_t noise, int32_t scheme, int32_t d, double *out)
{
    const int64_t V = volume(L);
    cplx *eta = (cplx *)out;
    const int tsrc = (int)(noise % L[3]);
#pragma omp parallel for schedule(static) if (V >= 1024)
    for (int64_t i = 0; i < V; ++i) {
        int c[4];
        coords(L, i, c);
        for (int al = 0; al < 4; ++al)
            for (int a = 0; a < 3; ++a) {
                cplx v = z2_entry(seed, V, noise, i, al, a);
                if (d >= 0 && or_dilution_class(L, scheme, i, al, a) != d) v = 0;
                if ((scheme & 64) && c[3] != tsrc) v = 0;
                eta[(i * 4 + al) * 3 + a] = v;
            }
    }
}

/* ------------------------------------------------------------------ */
/* Loop contraction (Section 3, zero-momentum local loop)              */
/* ------------------------------------------------------------------ */

/*
 * L[g][t] += sum_{x: x_4 = t} eta(x)^dagger Gamma_{gammas[g]} s(x),
 * spin and colour summed, L as [n_gamma][T][re,im].
 */
void or_loops_accumulate(const int32_t *L, const double *etad, const double *sd, int32_t n_gamma,
                         const int32_t *gammas, double *out)
{
    const cplx *eta = (const cplx *)etad, *s = (const cplx *)sd;
    const int64_t V = volume(L);
    const int T = L[3];
    for (int g = 0; g < n_gamma; ++g) {
        cplx G[4][4];
        gamma_n(gammas[g], G);
        for (int64_t i = 0; i < V; ++i) {
            int c[4];
            coords(L, i, c);
            cplx sum = 0;
            for (int al = 0; al < 4; ++al)
                for (int be = 0; be < 4; ++be)
                    for (int a = 0; a < 3; ++a) sum += conj(eta[(i * 4 + al) * 3 + a]) * G[al][be] * s[(i * 4 + be) * 3 + a];
            out[2 * (g * T + c[3])] += creal(sum);
            out[2 * (g * T + c[3]) + 1] += cimag(sum);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Link gradient of the loop estimator                                 */
/* ------------------------------------------------------------------ */

/*
 * For a real functional F = Re sum conj(W) L with the estimator
 * L = eta^+ P_t Gamma M^-1 eta and s = M^-1 eta, the variation is
 *   dF = Re kappa a^+ dD s,   a = M^-+ (sum W Gamma^+ P_t eta),
 * where a is passed in.  Accumulates into grad [4][V][3][3][re,im] the
 * derivative in the dF = Re(conj(g) dU) convention, from
 *   a(x)^+ (1 - g_mu) b dU_mu(x) s(x+mu)  and  a(x+mu)^+ (1 + g_mu) b dU_mu(x)^+ s(x).
 */
void or_link_grad_accumulate(const int32_t *L, int32_t tap, double kappa, const double *ad, const double *sd,
                             double *gradd)
{
    const cplx *a = (const cplx *)ad, *s = (const cplx *)sd;
    cplx *grad = (cplx *)gradd;
    const int64_t V = volume(L);
    cplx gam[4][4][4];
    for (int mu = 0; mu < 4; ++mu) gamma_mu(mu, gam[mu]);
#pragma omp parallel for schedule(static) if (V >= 1024)
    for (int64_t i = 0; i < V; ++i) {
        int c[4];
        coords(L, i, c);
        for (int mu = 0; mu < 4; ++mu) {
            const int64_t j = hop(L, i, mu, +1);
            const double b = bc_sign(L, tap, c, mu, +1);
            /* X_{ac} = sum_{al,be} conj(a_{al a}(x)) (1-g)_{al be} s_{be c}(x+mu)
               Y_{ac} = sum_{al,be} conj(a_{al a}(x+mu)) (1+g)_{al be} s_{be c}(x) */
            cplx X[3][3], Y[3][3];
            for (int aa = 0; aa < 3; ++aa)
                for (int cc = 0; cc < 3; ++cc) {
                    cplx sx = 0, sy = 0;
                    for (int al = 0; al < 4; ++al)
                        for (int be = 0; be < 4; ++be) {
                            cplx pm = (al == be ? 1.0 : 0.0) - gam[mu][al][be];
                            cplx pp = (al == be ? 1.0 : 0.0) + gam[mu][al][be];
                            sx += conj(a[(i * 4 + al) * 3 + aa]) * pm * s[(j * 4 + be) * 3 + cc];
                            sy += conj(a[(j * 4 + al) * 3 + aa]) * pp * s[(i * 4 + be) * 3 + cc];
                        }
                    X[aa][cc] = sx;
                    Y[aa][cc] = sy;
                }
            /* dF = Re k b sum_{ac} (X_ac dU_ac + Y_ca conj(dU_ac)) -> g_ac = k b (conj X_ac + Y_ca) */
            cplx *g = grad + (mu * V + i) * 9;
            for (int aa = 0; aa < 3; ++aa)
                for (int cc = 0; cc < 3; ++cc) g[3 * aa + cc] += kappa * b * (conj(X[aa][cc]) + Y[cc][aa]);
        }
    }
}

/* apply gamma_5 = diag(1,1,-1,-1) in place */
void or_gamma5(const int32_t *L, double *vd)
{
    cplx *v = (cplx *)vd;
    const int64_t V = volume(L);
    for (int64_t i = 0; i < V; ++i)
        for (int al = 2; al < 4; ++al)
            for (int a = 0; a < 3; ++a) v[(i * 4 + al) * 3 + a] = -v[(i * 4 + al) * 3 + a];
}

/*
 * out(x) = sum_g W[g][t(x)] Gamma_g^+ eta(x): the source of the adjoint
 * solve, W as [n_gamma][T][re,im].
 */
void or_weighted_gamma_dag(const int32_t *L, const double *etad, int32_t n_gamma, const int32_t *gammas,
                           const double *W, double *outd)
{
    const cplx *eta = (const cplx *)etad;
    cplx *out = (cplx *)outd;
    const int64_t V = volume(L);
    const int T = L[3];
    memset(out, 0, sizeof(cplx) * V * 12);
    for (int g = 0; g < n_gamma; ++g) {
        cplx G[4][4];
        gamma_n(gammas[g], G);
        for (int64_t i = 0; i < V; ++i) {
            int c[4];
            coords(L, i, c);
            cplx w = W[2 * (g * T + c[3])] + _Complex_I * W[2 * (g * T + c[3]) + 1];
            for (int al = 0; al < 4; ++al)
                for (int a = 0; a < 3; ++a) {
                    cplx sum = 0;
                    for (int be = 0; be < 4; ++be) sum += conj(G[be][al]) * eta[(i * 4 + be) * 3 + a];
                    out[(i * 4 + al) * 3 + a] += w * sum;
                }
        }
    }
}

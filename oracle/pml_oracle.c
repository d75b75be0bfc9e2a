/*
 * FP64 CPU oracle of the damped-current PML particle-in-cell step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * use it.  It shares no code, header, table or constant with the HIP library.
 *
 * The oracle is deliberately plain: absolute FP64 grid coordinates for particles,
 * all twelve split field parts stored everywhere (in the interior both parts of a
 * component are undamped, so only their sum matters), direct loops, no blocking or
 * fusion, compiled with -O2 -ffp-contract=off.  A second build of the same file with
 * -fopenmp (liboracle_omp.so) spreads the cell loops and the particle loop over the host's
 * cores, each thread depositing into its own current buffer, summed in thread order (a
 * fixed order for a given thread count); without -fopenmp the pragmas are ignored and the
 * particle loop below is the plain serial one.
 *
 * What it computes, and where each part comes from (Lehe et al., "Absorption of
 * charged particles in Perfectly-Matched-Layers by optimal damping of the deposited
 * current"):
 *   - split-field Maxwell equations with the damped current source: Sec. II.A,
 *     Eqs. (MaxwellE), (MaxwellB), (MaxwellSum), written for a PML normal along any
 *     axis (cyclic relabelling of the paper's z-face equations);
 *   - damping coefficient alpha = exp(-(1/v) int sigma/eps0): Sec. II.A, Eq. (alpha),
 *     evaluated at nodes and cell centres in closed form (Sec. II.B);
 *   - alpha = 0 (standard Berenger PML) and alpha = 1 (undamped deposition): the two
 *     comparison schemes of Sec. I / Fig. 1 caption;
 *   - Yee staggering and FDTD (Sec. II.B), 2D by dropping z derivatives (end of
 *     Sec. II.A);
 *   - Esirkepov charge-conserving deposition with B-spline shapes (App. A);
 *   - static opposite-charge partner at the initial position, E = B = 0 at t = 0
 *     (App. A.1);
 *   - energy-norm error integrand over physical cells (Sec. III, Eq. (error)).
 * Readings where the paper is silent (time discretisation of the PML terms, split
 * of the current in corners, alpha in corners, gather/push) are stated next to the
 * code that makes them.
 *
 * Units: c = eps0 = mu0 = 1.  Grid coordinates X are in node-index units; node i
 * along axis d sits at physical position (i - pml_lo[d]) * dx[d], so the physical
 * box is [0, n[d] dx[d]] and the PML lies outside it.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "pml_oracle.h"

#define NPART 12

/* ---------------------------------------------------------------- B-spline shapes */

/* Centred cardinal B-spline of degree `order` (1 linear, 2 quadratic, 3 cubic),
 * the particle shape factor of App. A (linear for the cavity runs, cubic "piecewise
 * cubic spline" for the single-particle runs).  Argument d is the distance from the
 * node in cell units. */
double orc_shape(int order, double d)
{
    double a = fabs(d);
    if (order == 1) {
        return a < 1.0 ? 1.0 - a : 0.0;
    } else if (order == 2) {
        if (a < 0.5) return 0.75 - a * a;
        if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
        return 0.0;
    } else if (order == 3) {
        if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
        if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
        return 0.0;
    }
    return 0.0;
}

/* ---------------------------------------------------------------- PML profiles */

/* Depth (physical length) of grid coordinate X inside the PML of axis d; 0 in the
 * physical box.  Also returns the thickness (physical length) of that side's PML. */
static double depth(const orc_sim *s, int d, double X, double *thick)
{
    double lo = (double)s->p.pml[d][0];
    double hi = (double)(s->p.pml[d][0] + s->p.n[d]);
    *thick = 0.0;
    if (d >= s->p.dim) return 0.0;
    if (X < lo) { *thick = s->p.pml[d][0] * s->p.dx[d]; return (lo - X) * s->p.dx[d]; }
    if (X > hi) { *thick = s->p.pml[d][1] * s->p.dx[d]; return (X - hi) * s->p.dx[d]; }
    return 0.0;
}

/* sigma/eps0 at depth delta: the graded profile sum_k a_k (delta/L)^k (the paper's
 * Eq. (conductivity) is the k = 2 member with a_2 = 4 (L/6)^2 / dx). */
static double sigma_of_depth(const orc_sim *s, int d, double delta, double L)
{
    if (delta <= 0.0 || L <= 0.0) return 0.0;
    double r = delta / L, acc = 0.0, pw = 1.0;
    for (int k = 0; k < s->p.n_sigma_coef; ++k) { acc += s->p.sigma_coef[d][k] * pw; pw *= r; }
    return acc;
}

/* Phi(delta) = int_0^delta sigma(z')/eps0 dz', exact integral of the polynomial. */
static double phi_of_depth(const orc_sim *s, int d, double delta, double L)
{
    if (delta <= 0.0 || L <= 0.0) return 0.0;
    double r = delta / L, acc = 0.0, pw = r;
    for (int k = 0; k < s->p.n_sigma_coef; ++k) {
        acc += s->p.sigma_coef[d][k] * L * pw / (double)(k + 1);
        pw *= r;
    }
    return acc;
}

double orc_sigma(const orc_sim *s, int d, double X)
{
    double L, del = depth(s, d, X, &L);
    return sigma_of_depth(s, d, del, L);
}

/* Eq. (alpha): alpha_d = exp(-(1/v) Phi_d), with damping_scale = 1/v (c = 1). */
double orc_alpha_axis(const orc_sim *s, int d, double X)
{
    double L, del = depth(s, d, X, &L);
    return exp(-s->p.damping_scale * phi_of_depth(s, d, del, L));
}

/* Mode of the layer that grid coordinate X lies in along axis d: the face's own mode
 * when one is set, else the global one.  Per-face modes are the combination the paper
 * proposes for a beam that enters through one PML and leaves through the other (end of
 * Sec. IV.A): undamped deposition (mode 1) where particles enter, Eq. (alpha) where
 * they leave. */
static int face_mode(const orc_sim *s, int d, double X)
{
    int side = X < (double)s->p.pml[d][0] ? 0 : 1;
    int f = s->p.alpha_face[d][side];
    return f > 0 ? f - 1 : s->p.alpha_mode;
}

/* Current-damping factor at a sample with grid coordinates X[3] (in-plane axes only).
 *   mode 0: alpha = 0 anywhere in the PML (standard Berenger PML, no source there);
 *   mode 1: alpha = 1 (undamped deposition);
 *   mode 2: Eq. (alpha); in edges and corners the product of the per-axis factors
 *           (reading: reduces to Eq. (alpha) on a face);
 *   mode 3: alpha = 1 in the field equations, each particle's weight damped instead
 *           (Sec. II.C, discussion of the velocity limitation; see path_sigma).
 * With per-face modes each axis contributes the factor of the face the sample lies in
 * (0, 1 or its exp(-Phi/v)), so a corner takes the product of its faces' factors. */
double orc_alpha(const orc_sim *s, const double X[3])
{
    if (s->p.alpha_mode == 3) return 1.0;
    double a = 1.0;
    for (int d = 0; d < s->p.dim; ++d) {
        double L, del = depth(s, d, X[d], &L);
        if (del <= 0.0) continue;
        int mode = face_mode(s, d, X[d]);
        if (mode == 0) return 0.0;
        if (mode == 2) a *= exp(-s->p.damping_scale * phi_of_depth(s, d, del, L));
    }
    return a;
}

/* Per-particle damping of the weight (Sec. II.C, discussion and limitations): the
 * weight becomes w exp(-Lambda), Lambda = int sigma(x(t))/eps0 dt over the time spent
 * in the layers (the sum over axes in edges and corners).  Over one move along a
 * straight line from X0 to X1 (grid coordinates) in time tau, with s the signed
 * distance into a face's layer, the integral is exactly
 *     tau (Phi(max(s1,0)) - Phi(max(s0,0))) / (s1 - s0),
 * or tau sigma(s0) when the coordinate does not change. */
static double path_sigma(const orc_sim *s, const double X0[3], const double X1[3], double tau)
{
    double acc = 0.0;
    for (int d = 0; d < s->p.dim; ++d) {
        double h = s->p.dx[d];
        double lo = (double)s->p.pml[d][0], hi = (double)(s->p.pml[d][0] + s->p.n[d]);
        double Llo = s->p.pml[d][0] * h, Lhi = s->p.pml[d][1] * h;
        double sl0 = (lo - X0[d]) * h, sl1 = (lo - X1[d]) * h;   /* into the low layer */
        double sh0 = (X0[d] - hi) * h, sh1 = (X1[d] - hi) * h;   /* into the high layer */
        if (X1[d] == X0[d]) {
            acc += tau * (sigma_of_depth(s, d, sl0, Llo) + sigma_of_depth(s, d, sh0, Lhi));
        } else {
            acc += tau * (phi_of_depth(s, d, sl1, Llo) - phi_of_depth(s, d, sl0, Llo)) / (sl1 - sl0);
            acc += tau * (phi_of_depth(s, d, sh1, Lhi) - phi_of_depth(s, d, sh0, Lhi)) / (sh1 - sh0);
        }
    }
    return acc;
}

/* a particle's weight with its damping (mode 3) */
static double particle_weight(const orc_sim *s, long t)
{
    return s->p.alpha_mode == 3 ? s->W[t] * exp(-s->LAM[t]) : s->W[t];
}

/* Lambda of the particles, in the order of orc_get_particles */
void orc_get_lambda(const orc_sim *s, double *lam)
{
    for (long t = 0; t < s->np; ++t) lam[t] = s->LAM[t];
}

double orc_path_sigma(const orc_sim *s, const double X0[3], const double X1[3], double tau)
{
    return path_sigma(s, X0, X1, tau);
}

/* Exponential time-differencing factors for dF/dt = -sig F + rhs over tau:
 * F <- e F + g rhs with e = exp(-sig tau), g = (1 - e)/sig (g = tau when sig = 0).
 * Reading of "the usual FDTD discretization" of Sec. II.B (Berenger's scheme). */
static void expfac(double sig, double tau, double *e, double *g)
{
    if (sig == 0.0) { *e = 1.0; *g = tau; return; }
    *e = exp(-sig * tau);
    *g = -expm1(-sig * tau) / sig;
}

/* ---------------------------------------------------------------- indexing */

static int nvalid(const orc_sim *s, int d, int stag)
{
    if (d >= s->p.dim) return 1;
    return s->M[d] + (stag ? 0 : 1);
}

/* component c: 0..2 = E_x,E_y,E_z ; 3..5 = B_x,B_y,B_z.  stagger along axis d. */
static int stag_of(int c, int d)
{
    int a = c % 3;
    if (c < 3) return d == a;   /* E_a: half-integer along a */
    return d != a;              /* B_a: half-integer across a */
}

static size_t idx3(const orc_sim *s, int i, int j, int k)
{
    return ((size_t)k * s->nn[1] + (size_t)j) * s->nn[0] + (size_t)i;
}

static int in_range(const orc_sim *s, int c, const int ii[3])
{
    for (int d = 0; d < 3; ++d) {
        if (ii[d] < 0 || ii[d] >= nvalid(s, d, stag_of(c, d))) return 0;
    }
    return 1;
}

static double total_at(const orc_sim *s, int c, const int ii[3])
{
    if (!in_range(s, c, ii)) return 0.0;
    size_t q = idx3(s, ii[0], ii[1], ii[2]);
    return s->F[2 * c][q] + s->F[2 * c + 1][q];
}

/* grid coordinate of sample ii of component c (J_a shares E_a's positions) */
static void sample_pos(int c, const int ii[3], double X[3])
{
    for (int d = 0; d < 3; ++d) X[d] = ii[d] + (stag_of(c, d) ? 0.5 : 0.0);
}

/* ---------------------------------------------------------------- lifecycle */

orc_sim *orc_create(const orc_params *p)
{
    if (p->dim != 2 && p->dim != 3) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->p = *p;
    for (int d = 0; d < 3; ++d) {
        if (d < p->dim) { s->M[d] = p->n[d] + p->pml[d][0] + p->pml[d][1]; s->nn[d] = s->M[d] + 1; }
        else { s->M[d] = 0; s->nn[d] = 1; }
    }
    s->nsamp = (size_t)s->nn[0] * s->nn[1] * s->nn[2];
    for (int q = 0; q < NPART; ++q) s->F[q] = (double *)calloc(s->nsamp, sizeof(double));
    for (int a = 0; a < 3; ++a) s->J[a] = (double *)calloc(s->nsamp, sizeof(double));
    s->rho_static = (double *)calloc(s->nsamp, sizeof(double));
    s->cap = 0; s->np = 0; s->next_id = 0;
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    for (int q = 0; q < NPART; ++q) free(s->F[q]);
    for (int a = 0; a < 3; ++a) free(s->J[a]);
    free(s->rho_static); free(s->X); free(s->U); free(s->W); free(s->LAM); free(s->id);
    free(s->cond); free(s->SX); free(s->SU); free(s->SW); free(s->sstep); free(s->sid);
    free(s->Jt);
    free(s);
}

size_t orc_num_samples(const orc_sim *s) { return s->nsamp; }
long orc_num_particles(const orc_sim *s) { return s->np; }
long orc_step_count(const orc_sim *s) { return s->step; }

static void reserve(orc_sim *s, long n)
{
    if (n <= s->cap) return;
    long c = s->cap ? s->cap : 16;
    while (c < n) c *= 2;
    s->X = (double *)realloc(s->X, sizeof(double) * 3 * c);
    s->U = (double *)realloc(s->U, sizeof(double) * 3 * c);
    s->W = (double *)realloc(s->W, sizeof(double) * c);
    s->LAM = (double *)realloc(s->LAM, sizeof(double) * c);
    s->id = (long *)realloc(s->id, sizeof(long) * c);
    s->cap = c;
}

/* charge density of one particle at the nodes, added with factor `sign` into rho */
static void deposit_rho(const orc_sim *s, const double X[3], double qw, double sign, double *rho)
{
    double dV = 1.0;
    for (int d = 0; d < s->p.dim; ++d) dV *= s->p.dx[d];
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < s->p.dim; ++d) { lo[d] = (int)floor(X[d]) - 3; hi[d] = (int)floor(X[d]) + 4; }
    for (int k = lo[2]; k <= hi[2]; ++k)
    for (int j = lo[1]; j <= hi[1]; ++j)
    for (int i = lo[0]; i <= hi[0]; ++i) {
        int ii[3] = {i, j, k};
        double w = 1.0;
        for (int d = 0; d < s->p.dim; ++d) w *= orc_shape(s->p.shape_order, X[d] - ii[d]);
        if (w == 0.0) continue;
        int ok = 1;
        for (int d = 0; d < 3; ++d) if (ii[d] < 0 || ii[d] >= s->nn[d]) ok = 0;
        if (!ok) continue;
        rho[idx3(s, i, j, k)] += sign * qw * w / dV;
    }
}

/* Adds particles given physical positions x (n x dim, origin at the physical-box
 * corner), momenta u = gamma v (n x 3) and weights w.  Each one also gets a
 * motionless opposite-charge partner at its initial position (App. A.1), which
 * enters only the charge density. */
int orc_add_particles(orc_sim *s, long n, const double *x, const double *u, const double *w)
{
    reserve(s, s->np + n);
    for (long t = 0; t < n; ++t) {
        long q = s->np++;
        for (int d = 0; d < 3; ++d) {
            s->X[3 * q + d] = d < s->p.dim ? x[s->p.dim * t + d] / s->p.dx[d] + s->p.pml[d][0] : 0.0;
            s->U[3 * q + d] = u[3 * t + d];
        }
        s->W[q] = w[t];
        s->LAM[q] = 0.0;
        s->id[q] = s->next_id++;
        deposit_rho(s, &s->X[3 * q], s->p.charge * w[t], -1.0, s->rho_static);
    }
    return 0;
}

/* Replaces the particle list (grid coordinates X, n x 3; ids given), without
 * touching the static partner density. */
int orc_set_particles(orc_sim *s, long n, const long *id, const double *X, const double *u, const double *w)
{
    s->np = 0;
    reserve(s, n);
    for (long t = 0; t < n; ++t) {
        for (int d = 0; d < 3; ++d) { s->X[3 * t + d] = X[3 * t + d]; s->U[3 * t + d] = u[3 * t + d]; }
        s->W[t] = w[t]; s->LAM[t] = 0.0; s->id[t] = id[t];
        if (id[t] >= s->next_id) s->next_id = id[t] + 1;
    }
    s->np = n;
    return 0;
}

void orc_get_particles(const orc_sim *s, long *id, double *X, double *u, double *w)
{
    for (long t = 0; t < s->np; ++t) {
        id[t] = s->id[t]; w[t] = s->W[t];
        for (int d = 0; d < 3; ++d) { X[3 * t + d] = s->X[3 * t + d]; u[3 * t + d] = s->U[3 * t + d]; }
    }
}

/* fields as 12 split parts, each nsamp doubles, order
 * E_xy E_xz E_yz E_yx E_zx E_zy B_xy B_xz B_yz B_yx B_zx B_zy */
void orc_get_fields(const orc_sim *s, double *out)
{
    for (int q = 0; q < NPART; ++q) memcpy(out + q * s->nsamp, s->F[q], sizeof(double) * s->nsamp);
}

void orc_set_fields(orc_sim *s, const double *in)
{
    for (int q = 0; q < NPART; ++q) memcpy(s->F[q], in + q * s->nsamp, sizeof(double) * s->nsamp);
}

void orc_get_current(const orc_sim *s, double *out)
{
    for (int a = 0; a < 3; ++a) memcpy(out + a * s->nsamp, s->J[a], sizeof(double) * s->nsamp);
}

void orc_get_rho_static(const orc_sim *s, double *out)
{
    memcpy(out, s->rho_static, sizeof(double) * s->nsamp);
}

void orc_set_rho_static(orc_sim *s, const double *in)
{
    memcpy(s->rho_static, in, sizeof(double) * s->nsamp);
}

/* ---------------------------------------------------------------- particles */

/* Field gather: each total component (sum of its split parts, Eq. (MaxwellSum)) at
 * grid position X, with the same-order B-spline at that component's staggered
 * sample positions.  Samples outside the grid (beyond the PEC walls) count as 0.
 * (Reading: the paper does not spell out the gather.) */
void orc_gather(const orc_sim *s, const double X[3], double EB[6])
{
    int m = s->p.shape_order;
    for (int c = 0; c < 6; ++c) {
        double acc = 0.0;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int d = 0; d < s->p.dim; ++d) { lo[d] = (int)floor(X[d]) - 3; hi[d] = (int)floor(X[d]) + 3; }
        for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
            int ii[3] = {i, j, k};
            double wgt = 1.0;
            for (int d = 0; d < s->p.dim; ++d)
                wgt *= orc_shape(m, X[d] - (ii[d] + (stag_of(c, d) ? 0.5 : 0.0)));
            if (wgt == 0.0) continue;
            acc += wgt * total_at(s, c, ii);
        }
        EB[c] = acc;
    }
}

/* Relativistic Boris rotation (Boris 1970), u = gamma v:
 * half electric kick, magnetic rotation, half electric kick. */
void orc_boris(double qdt_2m, const double E[3], const double B[3], double u[3])
{
    double um[3], t[3], up[3], sv[3], cr[3];
    for (int d = 0; d < 3; ++d) um[d] = u[d] + qdt_2m * E[d];
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int d = 0; d < 3; ++d) t[d] = qdt_2m * B[d] / gm;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int d = 0; d < 3; ++d) sv[d] = 2.0 * t[d] / (1.0 + t2);
    cr[0] = um[1] * t[2] - um[2] * t[1];
    cr[1] = um[2] * t[0] - um[0] * t[2];
    cr[2] = um[0] * t[1] - um[1] * t[0];
    for (int d = 0; d < 3; ++d) up[d] = um[d] + cr[d];
    cr[0] = up[1] * sv[2] - up[2] * sv[1];
    cr[1] = up[2] * sv[0] - up[0] * sv[2];
    cr[2] = up[0] * sv[1] - up[1] * sv[0];
    for (int d = 0; d < 3; ++d) u[d] = um[d] + cr[d] + qdt_2m * E[d];
}

static void add_J(orc_sim *s, int a, const int ii[3], double v, double *const J[3])
{
    if (!in_range(s, a, ii)) return;   /* guard samples beyond the walls are dropped */
    J[a][idx3(s, ii[0], ii[1], ii[2])] += v;
}

/* Esirkepov charge-conserving deposition (Esirkepov 2001, used in App. A) of one
 * particle of charge qw moving X0 -> X1 during dt, into J[3] (J_a at E_a's samples).
 * vz is its z velocity, used only in 2D (2D3V current along the invariant axis).
 *   2D: W_x = dSx (S0y + S1y)/2, W_y = dSy (S0x + S1x)/2,
 *       W_z = S0xS0y/3 + S1xS0y/6 + S0xS1y/6 + S1xS1y/3;
 *   3D: W_x = dSx (S0yS0z/3 + S1yS0z/6 + S0yS1z/6 + S1yS1z/3) and cyclic.
 * J_a(i_a + 1/2) - J_a(i_a - 1/2) = -qw W_a / (dt * product of the other dx),
 * accumulated from zero at the low end of the stencil. */
void orc_deposit(orc_sim *s, const double X0[3], const double X1[3], double vz, double qw, double *const J[3])
{
    int dim = s->p.dim, m = s->p.shape_order;
    enum { WN = 12 };
    int lo[3] = {0, 0, 0}, n[3] = {1, 1, 1};
    double S0[3][WN], S1[3][WN], DS[3][WN];
    for (int d = 0; d < 3; ++d) {
        for (int t = 0; t < WN; ++t) { S0[d][t] = 1.0; S1[d][t] = 1.0; DS[d][t] = 0.0; }
    }
    for (int d = 0; d < dim; ++d) {
        double mn = X0[d] < X1[d] ? X0[d] : X1[d];
        double mx = X0[d] < X1[d] ? X1[d] : X0[d];
        lo[d] = (int)floor(mn) - 3;
        n[d] = (int)floor(mx) + 4 - lo[d] + 1;
        if (n[d] > WN) n[d] = WN;  /* moves are below one cell per step */
        for (int t = 0; t < n[d]; ++t) {
            S0[d][t] = orc_shape(m, X0[d] - (lo[d] + t));
            S1[d][t] = orc_shape(m, X1[d] - (lo[d] + t));
            DS[d][t] = S1[d][t] - S0[d][t];
        }
    }
    double dV = 1.0;
    for (int d = 0; d < dim; ++d) dV *= s->p.dx[d];
    double dt = s->p.dt;
    if (dim == 2) {
        double cx = qw / (s->p.dx[1] * dt), cy = qw / (s->p.dx[0] * dt);
        for (int tj = 0; tj < n[1]; ++tj) {           /* J_x: running sum along x */
            double acc = 0.0;
            for (int ti = 0; ti < n[0]; ++ti) {
                double Wx = 0.5 * DS[0][ti] * (S0[1][tj] + S1[1][tj]);
                acc -= cx * Wx;
                int ii[3] = {lo[0] + ti, lo[1] + tj, 0};
                if (acc != 0.0) add_J(s, 0, ii, acc, J);
            }
        }
        for (int ti = 0; ti < n[0]; ++ti) {           /* J_y: running sum along y */
            double acc = 0.0;
            for (int tj = 0; tj < n[1]; ++tj) {
                double Wy = 0.5 * DS[1][tj] * (S0[0][ti] + S1[0][ti]);
                acc -= cy * Wy;
                int ii[3] = {lo[0] + ti, lo[1] + tj, 0};
                if (acc != 0.0) add_J(s, 1, ii, acc, J);
            }
        }
        for (int tj = 0; tj < n[1]; ++tj)              /* J_z: path-averaged shape */
        for (int ti = 0; ti < n[0]; ++ti) {
            double Wz = S0[0][ti] * S0[1][tj] / 3.0 + S1[0][ti] * S0[1][tj] / 6.0
                      + S0[0][ti] * S1[1][tj] / 6.0 + S1[0][ti] * S1[1][tj] / 3.0;
            if (Wz == 0.0) continue;
            int ii[3] = {lo[0] + ti, lo[1] + tj, 0};
            add_J(s, 2, ii, qw * vz * Wz / dV, J);
        }
    } else {
        for (int a = 0; a < 3; ++a) {
            int b = (a + 1) % 3, c = (a + 2) % 3;
            double coef = qw / (s->p.dx[b] * s->p.dx[c] * dt);
            for (int tc = 0; tc < n[c]; ++tc)
            for (int tb = 0; tb < n[b]; ++tb) {
                double avg = S0[b][tb] * S0[c][tc] / 3.0 + S1[b][tb] * S0[c][tc] / 6.0
                           + S0[b][tb] * S1[c][tc] / 6.0 + S1[b][tb] * S1[c][tc] / 3.0;
                double acc = 0.0;
                for (int ta = 0; ta < n[a]; ++ta) {
                    acc -= coef * DS[a][ta] * avg;
                    int ii[3];
                    ii[a] = lo[a] + ta; ii[b] = lo[b] + tb; ii[c] = lo[c] + tc;
                    if (acc != 0.0) add_J(s, a, ii, acc, J);
                }
            }
        }
    }
}

/* ---------------------------------------------------------------- fields */

/* Levi-Civita symbol for a permutation of (0,1,2) */
static int levi(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0;
    return ((a + 1) % 3 == b) ? 1 : -1;
}

/* Fraction of J_a that enters split part E_ab (derivative axis b; c the third axis).
 * The paper's z-face equations put the whole current of the transverse components
 * into the part damped by sigma_z and the longitudinal one into the (undamped)
 * E_z.  Reading for every face, edge and corner: weight sigma_b/(sigma_b+sigma_c);
 * where both vanish the whole current goes to the part with b = a+1 (mod 3); there
 * both parts are undamped, so only their sum matters.  Pins: the exit-error ordering at
 * 60 degrees (a transverse current in the undamped part breaks it) and the x-y mirror
 * symmetry of an edge and corner run; parity unpinned beyond them (another rule that is
 * symmetric in b and c and equals the face assignment would pass both). */
static double source_weight(int a, int b, double sb, double sc)
{
    if (sb + sc > 0.0) return sb / (sb + sc);
    return (b == (a + 1) % 3) ? 1.0 : 0.0;
}

/* Advance every split part of E (is_e = 1, with the damped current) or B (is_e = 0)
 * by tau.  For part F_ab of component a (b the derivative axis):
 *   dE_ab/dt =  eps_abc d_b B_c - sigma_b E_ab - w_ab alpha J_a    (Eq. MaxwellE)
 *   dB_ab/dt = -eps_abc d_b E_c - sigma_b B_ab                     (Eq. MaxwellB)
 * with sigma_b taken at the sample's coordinate along b, integrated with the
 * exponential factors of expfac().  In 2D the z derivatives vanish. */
/* Cole-Karkkainen difference (App. A: the paper's solver, with cubic cells) of E
 * component ci along b, at the B sample ii: the Yee difference E(ii + e_b) - E(ii) at ii
 * and at its transverse neighbours, weighted 7/12 at ii, 1/12 at each of the four side
 * neighbours and 1/48 at each of the four diagonal ones (weights sum to 1, so a field
 * uniform across b gives the Yee difference: no dispersion along the axes at c dt = dx).
 * Used for Faraday's law only; Ampere's law keeps the Yee difference. */
static double ck_diff(const orc_sim *s, int ci, const int ii[3], int b)
{
    int t1 = (b + 1) % 3, t2 = (b + 2) % 3;
    double acc = 0.0;
    for (int o1 = -1; o1 <= 1; ++o1)
        for (int o2 = -1; o2 <= 1; ++o2) {
            int nside = (o1 != 0) + (o2 != 0);
            double w = nside == 0 ? 7.0 / 12.0 : (nside == 1 ? 1.0 / 12.0 : 1.0 / 48.0);
            int p[3] = {ii[0], ii[1], ii[2]};
            p[t1] += o1;
            p[t2] += o2;
            int q[3] = {p[0], p[1], p[2]};
            q[b] += 1;
            acc += w * (total_at(s, ci, q) - total_at(s, ci, p));
        }
    return acc;
}

/* Binomial filter of the deposited current (App. A): J_a <- sum over the 3^dim
 * neighbours o of prod_d (1/4, 1/2, 1/4)[o_d] J_a(ii + o), once per pass; samples outside
 * J_a's extent count as zero and are not written. */
void orc_filter_current(orc_sim *s)
{
    int dim = s->p.dim;
    double *tmp = (double *)calloc(s->nsamp, sizeof(double));
    for (int pass = 0; pass < s->p.filter_passes; ++pass)
        for (int a = 0; a < 3; ++a) {
            int nv[3];
            for (int d = 0; d < 3; ++d) nv[d] = nvalid(s, d, stag_of(a, d));
            #pragma omp parallel for collapse(2) schedule(static)
            for (int k = 0; k < nv[2]; ++k)
            for (int j = 0; j < nv[1]; ++j)
            for (int i = 0; i < nv[0]; ++i) {
                double acc = 0.0;
                for (int oz = (dim == 3 ? -1 : 0); oz <= (dim == 3 ? 1 : 0); ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int p[3] = {i + ox, j + oy, k + oz};
                    if (!in_range(s, a, p)) continue;
                    double w = (ox ? 0.25 : 0.5) * (oy ? 0.25 : 0.5) * (dim == 3 ? (oz ? 0.25 : 0.5) : 1.0);
                    acc += w * s->J[a][idx3(s, p[0], p[1], p[2])];
                }
                tmp[idx3(s, i, j, k)] = acc;
            }
            for (int k = 0; k < nv[2]; ++k)
            for (int j = 0; j < nv[1]; ++j)
            for (int i = 0; i < nv[0]; ++i) s->J[a][idx3(s, i, j, k)] = tmp[idx3(s, i, j, k)];
        }
    free(tmp);
}

/* ---------------------------------------------------------------- conductors */

/* Conductor cells (the cavity run of App. A.2 models the cavity walls by setting E and B
 * to zero in the cells the walls cover).  Reading: a field sample is held at zero when it
 * lies in the closed extent of any conductor cell, i.e. along each axis the one cell it is
 * inside (half-integer coordinate) or the two cells it borders (integer coordinate).  On a
 * wall between a vacuum cell and a conductor cell this zeroes the tangential E and the
 * normal B, the perfect-conductor conditions of the staircase wall. */
int orc_sample_in_conductor(const orc_sim *s, int c, int i, int j, int k)
{
    if (!s->cond) return 0;
    int ii[3] = {i, j, k}, lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        if (stag_of(c, d)) { lo[d] = ii[d]; hi[d] = ii[d]; }
        else { lo[d] = ii[d] - 1; hi[d] = ii[d]; }
        if (lo[d] < 0) lo[d] = 0;
        if (hi[d] > s->M[d] - 1) hi[d] = s->M[d] - 1;
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y)
    for (int x = lo[0]; x <= hi[0]; ++x)
        if (s->cond[((size_t)z * s->M[1] + y) * s->M[0] + x]) return 1;
    return 0;
}

/* zeroes both split parts of every field sample inside a conductor */
static void apply_conductor(orc_sim *s)
{
    if (!s->cond) return;
    for (int c = 0; c < 6; ++c) {
        int nv[3];
        for (int d = 0; d < 3; ++d) nv[d] = nvalid(s, d, stag_of(c, d));
        for (int k = 0; k < nv[2]; ++k)
        for (int j = 0; j < nv[1]; ++j)
        for (int i = 0; i < nv[0]; ++i)
            if (orc_sample_in_conductor(s, c, i, j, k)) {
                size_t q = idx3(s, i, j, k);
                s->F[2 * c][q] = 0.0;
                s->F[2 * c + 1][q] = 0.0;
            }
    }
}

/* Sets the conductor cells (3D only; NULL removes them) and zeroes the fields inside. */
int orc_set_conductor(orc_sim *s, const unsigned char *cells)
{
    if (s->p.dim != 3) return -1;
    free(s->cond);
    s->cond = NULL;
    if (!cells) return 0;
    size_t nc = (size_t)s->M[0] * s->M[1] * s->M[2];
    s->cond = (unsigned char *)malloc(nc);
    memcpy(s->cond, cells, nc);
    apply_conductor(s);
    return 0;
}

static void advance(orc_sim *s, int is_e, double tau)
{
    for (int a = 0; a < 3; ++a) {
        int c_self = is_e ? a : 3 + a;
        for (int side = 0; side < 2; ++side) {
            int b = (a + 1 + side) % 3;        /* derivative axis of this part */
            int c = 3 - a - b;                 /* the other field's component */
            int ci = is_e ? 3 + c : c;         /* B_c for E parts, E_c for B parts */
            double eps = (double)levi(a, b, c);
            double *Fp = s->F[2 * c_self + side];
            int nv[3];
            for (int d = 0; d < 3; ++d) nv[d] = nvalid(s, d, stag_of(c_self, d));
            #pragma omp parallel for collapse(2) schedule(static)
            for (int k = 0; k < nv[2]; ++k)
            for (int j = 0; j < nv[1]; ++j)
            for (int i = 0; i < nv[0]; ++i) {
                int ii[3] = {i, j, k};
                if (is_e) {   /* PEC: tangential E on the outer walls stays 0 */
                    int on_wall = 0;
                    for (int d = 0; d < s->p.dim; ++d)
                        if (d != a && (ii[d] == 0 || ii[d] == s->M[d])) on_wall = 1;
                    if (on_wall) continue;
                }
                double X[3];
                sample_pos(c_self, ii, X);
                double deriv = 0.0;
                if (b < s->p.dim && !is_e && s->p.solver == 1) {
                    deriv = ck_diff(s, ci, ii, b) / s->p.dx[b];
                } else if (b < s->p.dim) {
                    int ip[3] = {i, j, k}, im[3] = {i, j, k};
                    if (is_e) { im[b] -= 1; }  /* B_c sits half a cell off along b */
                    else { ip[b] += 1; }       /* E_c sits half a cell off along b */
                    deriv = (total_at(s, ci, ip) - total_at(s, ci, im)) / s->p.dx[b];
                }
                double sb = orc_sigma(s, b, X[b]);
                double e, g;
                expfac(sb, tau, &e, &g);
                size_t q = idx3(s, i, j, k);
                double rhs = (is_e ? eps : -eps) * deriv;
                if (is_e) {
                    double sc = orc_sigma(s, c, X[c]);
                    double w = source_weight(a, b, sb, sc);
                    rhs -= w * s->J[a][q];    /* J already multiplied by alpha */
                }
                Fp[q] = e * Fp[q] + g * rhs;
            }
        }
    }
    apply_conductor(s);
}

/* J_a <- alpha J_a at J_a's samples (Eq. MaxwellE source term alpha j). */
static void damp_current(orc_sim *s)
{
    for (int a = 0; a < 3; ++a) {
        int nv[3];
        for (int d = 0; d < 3; ++d) nv[d] = nvalid(s, d, stag_of(a, d));
        #pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nv[2]; ++k)
        for (int j = 0; j < nv[1]; ++j)
        for (int i = 0; i < nv[0]; ++i) {
            int ii[3] = {i, j, k};
            double X[3];
            sample_pos(a, ii, X);
            s->J[a][idx3(s, i, j, k)] *= orc_alpha(s, X);
        }
    }
}

/* public single-phase entry points, for unit pins */
void orc_damp_current(orc_sim *s) { damp_current(s); }
void orc_advance_B(orc_sim *s, double tau) { advance(s, 0, tau); }
void orc_advance_E(orc_sim *s, double tau) { advance(s, 1, tau); }
void orc_zero_current(orc_sim *s) { for (int a = 0; a < 3; ++a) memset(s->J[a], 0, sizeof(double) * s->nsamp); }
void orc_set_current(orc_sim *s, const double *in)
{
    for (int a = 0; a < 3; ++a) memcpy(s->J[a], in + a * s->nsamp, sizeof(double) * s->nsamp);
}
void orc_deposit_into(orc_sim *s, const double X0[3], const double X1[3], double vz, double qw)
{
    orc_deposit(s, X0, X1, vz, qw, s->J);
}

/* ---------------------------------------------------------------- beam source */

/* Beam source (the cavity run of Sec. IV.A: a long beam injected continuously on one side
 * of the box, through that side's PML).  Each particle is given at the present time by its
 * physical position x (dim values), momentum u = gamma v and weight w, and moves
 * ballistically until the first step start t = (step + m) dt, m >= 0, at which its
 * position x + m dt v lies at or beyond the outer wall of the low layer of `axis`; it is
 * added then, at that position (so its first move starts inside the box), with no static
 * partner.  Ids follow the given order after those already assigned.  Fails (-1) for a
 * particle that never reaches the box or reaches it outside the box along another axis. */
int orc_set_source(orc_sim *s, long n, const double *x, const double *u, const double *w, int axis)
{
    int dim = s->p.dim;
    if (axis < 0 || axis >= dim) return -1;
    free(s->SX); free(s->SU); free(s->SW); free(s->sstep); free(s->sid);
    s->SX = (double *)malloc(sizeof(double) * 3 * (n + 1));
    s->SU = (double *)malloc(sizeof(double) * 3 * (n + 1));
    s->SW = (double *)malloc(sizeof(double) * (n + 1));
    s->sstep = (long *)malloc(sizeof(long) * (n + 1));
    s->sid = (long *)malloc(sizeof(long) * (n + 1));
    s->nsrc = 0;
    s->src_next = 0;
    double wall = -(double)s->p.pml[axis][0] * s->p.dx[axis];
    s->next_id += n;
    for (long t = 0; t < n; ++t) {
        const double *ut = u + 3 * t;
        double gam = sqrt(1.0 + ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
        double va = ut[axis] / gam;
        double xa = x[dim * t + axis];
        long m = 0;
        if (xa < wall) {
            if (!(va > 0.0)) { s->nsrc = 0; return -1; }
            m = (long)ceil((wall - xa) / (va * s->p.dt));
            if (m < 1) m = 1;
            while (xa + (double)m * s->p.dt * va < wall) ++m;
            while (m > 1 && xa + (double)(m - 1) * s->p.dt * va >= wall) --m;
        }
        long q = s->nsrc++;
        for (int d = 0; d < 3; ++d) {
            double Xd = 0.0;
            if (d < dim) {
                double xd = x[dim * t + d] + (double)m * s->p.dt * (ut[d] / gam);
                Xd = xd / s->p.dx[d] + s->p.pml[d][0];
                if (!(Xd >= 0.0 && Xd < (double)s->M[d])) { s->nsrc = 0; return -1; }
            }
            s->SX[3 * q + d] = Xd;
            s->SU[3 * q + d] = ut[d];
        }
        s->SW[q] = w[t];
        s->sstep[q] = s->step + m;
        s->sid[q] = s->next_id - n + t;
    }
    return 0;
}

/* adds the source particles whose injection step is the present one */
static void inject(orc_sim *s)
{
    for (long q = 0; q < s->nsrc; ++q) {
        if (s->sstep[q] != s->step) continue;
        reserve(s, s->np + 1);
        long t = s->np++;
        for (int d = 0; d < 3; ++d) { s->X[3 * t + d] = s->SX[3 * q + d]; s->U[3 * t + d] = s->SU[3 * q + d]; }
        s->W[t] = s->SW[q];
        s->LAM[t] = 0.0;
        s->id[t] = s->sid[q];
    }
}

/* One PIC step: E^n, B^n, X^n, u^{n-1/2}  ->  E^{n+1}, B^{n+1}, X^{n+1}, u^{n+1/2}.
 *  0. source particles due at t^n are added (beam source, see orc_set_source);
 *  1. per particle: gather E^n, B^n at X^n (totals), Boris push (if enabled),
 *     X^{n+1} = X^n + dt u/gamma, Esirkepov deposit of X^n -> X^{n+1};
 *     particles ending outside the PEC box are removed after depositing;
 *  2. J <- alpha J (Eq. alpha / mode), after the binomial filter when it is on;
 *  3. B += dt/2 from E^n; E += dt from B^{n+1/2} and alpha J; B += dt/2 from E^{n+1};
 *     after each of the three, samples inside conductor cells are set to zero. */
/* Particle t of step 1 below: gather, push, move to X1, deposit into J; updates u in
 * place and returns the new Lambda in *lam; returns 1 if it ends outside the PEC box. */
static int move_one(orc_sim *s, long t, double qdt_2m, double X1[3], double *lam, double *const J[3])
{
    int dim = s->p.dim;
    double *X = &s->X[3 * t], *u = &s->U[3 * t];
    if (s->p.push) {
        double EB[6];
        orc_gather(s, X, EB);
        orc_boris(qdt_2m, EB, EB + 3, u);
    }
    double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; ++d) X1[d] = X[d];
    for (int d = 0; d < dim; ++d) X1[d] = X[d] + s->p.dt * u[d] / gam / s->p.dx[d];
    double qw = s->p.charge * s->W[t];
    *lam = s->LAM[t];
    if (s->p.alpha_mode == 3) {
        /* weight damped by Lambda at mid-step (the time of the deposited current) */
        double Xh[3] = {X[0], X[1], X[2]};
        for (int d = 0; d < dim; ++d) Xh[d] = 0.5 * (X[d] + X1[d]);
        qw *= exp(-(*lam + path_sigma(s, X, Xh, 0.5 * s->p.dt)));
        *lam += path_sigma(s, X, X1, s->p.dt);
    }
    orc_deposit(s, X, X1, u[2] / gam, qw, J);
    int out = 0;
    for (int d = 0; d < dim; ++d) if (X1[d] < 0.0 || X1[d] >= (double)s->M[d]) out = 1;
    return out;
}

#ifdef _OPENMP
/* Step 1 over all cores: particles split statically over the threads, each depositing
 * into its own current buffer; the buffers are summed sample by sample in thread order;
 * then the survivors are compacted in their order. */
static void move_all_threads(orc_sim *s, double qdt_2m)
{
    int nthr = omp_get_max_threads();
    size_t ns = s->nsamp;
    if (s->nthr != nthr) {
        free(s->Jt);
        s->Jt = (double *)malloc(sizeof(double) * 3 * ns * (size_t)nthr);
        s->nthr = nthr;
    }
    long np = s->np;
    double *Xn = (double *)malloc(sizeof(double) * 3 * (np + 1));
    double *Ln = (double *)malloc(sizeof(double) * (np + 1));
    char *gone = (char *)malloc((size_t)np + 1);
    #pragma omp parallel num_threads(nthr)
    {
        int th = omp_get_thread_num();
        double *Jt[3];
        for (int a = 0; a < 3; ++a) {
            Jt[a] = s->Jt + ((size_t)th * 3 + a) * ns;
            memset(Jt[a], 0, sizeof(double) * ns);
        }
        #pragma omp for schedule(static)
        for (long t = 0; t < np; ++t) gone[t] = (char)move_one(s, t, qdt_2m, &Xn[3 * t], &Ln[t], Jt);
        #pragma omp for schedule(static)
        for (long q = 0; q < (long)ns; ++q)
            for (int a = 0; a < 3; ++a) {
                double acc = s->J[a][q];
                for (int u = 0; u < nthr; ++u) acc += s->Jt[((size_t)u * 3 + a) * ns + q];
                s->J[a][q] = acc;
            }
    }
    long keep = 0;
    for (long t = 0; t < np; ++t) {
        if (gone[t]) continue;
        for (int d = 0; d < 3; ++d) { s->X[3 * keep + d] = Xn[3 * t + d]; s->U[3 * keep + d] = s->U[3 * t + d]; }
        s->W[keep] = s->W[t]; s->LAM[keep] = Ln[t]; s->id[keep] = s->id[t];
        ++keep;
    }
    s->np = keep;
    free(Xn); free(Ln); free(gone);
}
#endif

void orc_step(orc_sim *s, int nsteps)
{
    double qdt_2m = s->p.charge * s->p.dt / (2.0 * s->p.mass);
    for (int it = 0; it < nsteps; ++it) {
        inject(s);
        orc_zero_current(s);
#ifdef _OPENMP
        move_all_threads(s, qdt_2m);
#else
        long keep = 0;
        for (long t = 0; t < s->np; ++t) {
            double X1[3], lam;
            if (move_one(s, t, qdt_2m, X1, &lam, s->J)) continue;
            for (int d = 0; d < 3; ++d) { s->X[3 * keep + d] = X1[d]; s->U[3 * keep + d] = s->U[3 * t + d]; }
            s->W[keep] = s->W[t]; s->LAM[keep] = lam; s->id[keep] = s->id[t];
            ++keep;
        }
        s->np = keep;
#endif
        if (s->p.filter_passes > 0) orc_filter_current(s);
        damp_current(s);
        advance(s, 0, 0.5 * s->p.dt);
        advance(s, 1, s->p.dt);
        advance(s, 0, 0.5 * s->p.dt);
        s->step++;
    }
}

/* ---------------------------------------------------------------- diagnostics */

static int in_physical(const orc_sim *s, const double X[3])
{
    for (int d = 0; d < s->p.dim; ++d) {
        if (X[d] < (double)s->p.pml[d][0] || X[d] > (double)(s->p.pml[d][0] + s->p.n[d])) return 0;
    }
    return 1;
}

/* out[0] U over samples in the physical box, out[1] U over the other samples,
 * out[2] max |div E - rho| and out[3] its RMS over interior nodes (strictly inside
 * the physical box), out[4] max |rho of the moving particles|, out[5] particle
 * count, out[6] step.  U = 1/2 sum (E^2 + B^2) dV over each component's samples. */
void orc_diagnose(const orc_sim *s, double out[7])
{
    double dV = 1.0;
    for (int d = 0; d < s->p.dim; ++d) dV *= s->p.dx[d];
    double ui = 0.0, up = 0.0;
    for (int c = 0; c < 6; ++c) {
        int nv[3];
        for (int d = 0; d < 3; ++d) nv[d] = nvalid(s, d, stag_of(c, d));
        for (int k = 0; k < nv[2]; ++k)
        for (int j = 0; j < nv[1]; ++j)
        for (int i = 0; i < nv[0]; ++i) {
            int ii[3] = {i, j, k};
            double X[3], v = total_at(s, c, ii);
            sample_pos(c, ii, X);
            if (in_physical(s, X)) ui += 0.5 * v * v * dV; else up += 0.5 * v * v * dV;
        }
    }
    double *rho = (double *)calloc(s->nsamp, sizeof(double));
    for (long t = 0; t < s->np; ++t) deposit_rho(s, &s->X[3 * t], s->p.charge * particle_weight(s, t), 1.0, rho);
    double rmax = 0.0;
    for (size_t q = 0; q < s->nsamp; ++q) if (fabs(rho[q]) > rmax) rmax = fabs(rho[q]);
    double gmax = 0.0, gsum = 0.0;
    long cnt = 0;
    for (int k = 0; k < s->nn[2]; ++k)
    for (int j = 0; j < s->nn[1]; ++j)
    for (int i = 0; i < s->nn[0]; ++i) {
        int ii[3] = {i, j, k};
        int inner = 1;
        for (int d = 0; d < s->p.dim; ++d)
            if (ii[d] <= s->p.pml[d][0] || ii[d] >= s->p.pml[d][0] + s->p.n[d]) inner = 0;
        if (!inner) continue;
        double div = 0.0;
        for (int d = 0; d < s->p.dim; ++d) {
            int im[3] = {i, j, k};
            im[d] -= 1;
            div += (total_at(s, d, ii) - total_at(s, d, im)) / s->p.dx[d];
        }
        size_t q = idx3(s, i, j, k);
        double r = div - rho[q] - s->rho_static[q];
        if (fabs(r) > gmax) gmax = fabs(r);
        gsum += r * r;
        ++cnt;
    }
    free(rho);
    out[0] = ui; out[1] = up; out[2] = gmax; out[3] = cnt ? sqrt(gsum / cnt) : 0.0;
    out[4] = rmax; out[5] = (double)s->np; out[6] = (double)s->step;
}

/* charge density of the current particles (without the static partners) */
void orc_rho(const orc_sim *s, double *rho)
{
    memset(rho, 0, sizeof(double) * s->nsamp);
    for (long t = 0; t < s->np; ++t) deposit_rho(s, &s->X[3 * t], s->p.charge * particle_weight(s, t), 1.0, rho);
}

/* Beam moments per slab along `axis` (the deflection diagnostic of Sec. IV.A, the change
 * of <u_x> = <p_x>/mc between planes): for slab k = [edges[k], edges[k+1]) in physical
 * coordinates, out[5k .. 5k+4] = (number of particles, sum w, sum w u_x, sum w u_y,
 * sum w u_z) over the particles whose position lies in it. */
void orc_slab_moments(const orc_sim *s, int axis, int nslab, const double *edges, double *out)
{
    for (int k = 0; k < 5 * nslab; ++k) out[k] = 0.0;
    for (long t = 0; t < s->np; ++t) {
        double xa = (s->X[3 * t + axis] - s->p.pml[axis][0]) * s->p.dx[axis];
        for (int k = 0; k < nslab; ++k) {
            if (xa >= edges[k] && xa < edges[k + 1]) {
                double w = s->W[t];
                out[5 * k + 0] += 1.0;
                out[5 * k + 1] += w;
                for (int d = 0; d < 3; ++d) out[5 * k + 2 + d] += w * s->U[3 * t + d];
                break;
            }
        }
    }
}

/*
 * FP64 CPU oracle of the damped-current PML particle-in-cell step.
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.  This header is the
 * oracle's own and is not included by any HIP source.
 */
#ifndef PML_ORACLE_H
#define PML_ORACLE_H
#include <stddef.h>

typedef struct {
    int dim;                 /* 2 (x-y plane, 2D3V) or 3 */
    int n[3];                /* physical cells per axis */
    int pml[3][2];           /* PML cells per axis, low / high side */
    double dx[3];
    double dt;
    int shape_order;         /* 1, 2, 3 */
    int alpha_mode;          /* 0: alpha = 0, 1: alpha = 1, 2: Eq. (alpha), 3: weights damped */
    double damping_scale;    /* 1/v of Eq. (alpha) */
    int n_sigma_coef;
    double sigma_coef[3][16];/* sigma_d/eps0 = sum_k coef[d][k] (depth/L)^k */
    int push;                /* 1: gather + Boris; 0: momenta kept (ballistic) */
    double charge, mass;     /* per unit weight */
    int solver;              /* 0: Yee; 1: Cole-Karkkainen in Faraday's law (3D, cubic cells) */
    int filter_passes;       /* binomial passes over the deposited current (0: none) */
    int alpha_face[3][2];    /* per-face alpha mode, low / high side: 0 = alpha_mode,
                                else 1 + mode (modes 0, 1, 2 only) */
} orc_params;

typedef struct {
    orc_params p;
    int M[3];                /* cells per axis incl. PML (0 for the invariant axis) */
    int nn[3];               /* nodes per axis (1 for the invariant axis) */
    size_t nsamp;
    double *F[12];           /* split parts, see orc_get_fields */
    double *J[3];
    double *rho_static;
    long np, cap, next_id;
    double *X, *U, *W;       /* grid coordinates (np x 3), u = gamma v (np x 3), weights */
    double *LAM;             /* mode 3: int sigma/eps0 dt along each particle's path */
    long *id;
    long step;
    unsigned char *cond;     /* conductor cells (M0 x M1 x M2, x fastest), NULL if none */
    long nsrc, src_next;     /* beam source: entries sorted by injection step */
    double *SX, *SU, *SW;    /* grid coordinates at injection, u, w */
    long *sstep, *sid;
    double *Jt;              /* all-cores build: per-thread current buffers (3 nsamp each) */
    int nthr;                /* threads they were allocated for */
} orc_sim;

double orc_shape(int order, double d);
double orc_sigma(const orc_sim *s, int d, double X);
double orc_alpha_axis(const orc_sim *s, int d, double X);
double orc_alpha(const orc_sim *s, const double X[3]);
orc_sim *orc_create(const orc_params *p);
void orc_destroy(orc_sim *s);
size_t orc_num_samples(const orc_sim *s);
long orc_num_particles(const orc_sim *s);
long orc_step_count(const orc_sim *s);
int orc_add_particles(orc_sim *s, long n, const double *x, const double *u, const double *w);
int orc_set_particles(orc_sim *s, long n, const long *id, const double *X, const double *u, const double *w);
void orc_get_particles(const orc_sim *s, long *id, double *X, double *u, double *w);
void orc_get_fields(const orc_sim *s, double *out);
void orc_set_fields(orc_sim *s, const double *in);
void orc_get_current(const orc_sim *s, double *out);
void orc_set_current(orc_sim *s, const double *in);
void orc_get_rho_static(const orc_sim *s, double *out);
void orc_set_rho_static(orc_sim *s, const double *in);
void orc_gather(const orc_sim *s, const double X[3], double EB[6]);
void orc_filter_current(orc_sim *s);
void orc_boris(double qdt_2m, const double E[3], const double B[3], double u[3]);
void orc_deposit(orc_sim *s, const double X0[3], const double X1[3], double vz, double qw, double *const J[3]);
void orc_deposit_into(orc_sim *s, const double X0[3], const double X1[3], double vz, double qw);
void orc_zero_current(orc_sim *s);
void orc_damp_current(orc_sim *s);
void orc_advance_B(orc_sim *s, double tau);
void orc_advance_E(orc_sim *s, double tau);
void orc_step(orc_sim *s, int nsteps);
void orc_diagnose(const orc_sim *s, double out[7]);
void orc_rho(const orc_sim *s, double *rho);
void orc_get_lambda(const orc_sim *s, double *lam);
double orc_path_sigma(const orc_sim *s, const double X0[3], const double X1[3], double tau);
int orc_set_conductor(orc_sim *s, const unsigned char *cells);
int orc_sample_in_conductor(const orc_sim *s, int c, int i, int j, int k);
int orc_set_source(orc_sim *s, long n, const double *x, const double *u, const double *w, int axis);
void orc_slab_moments(const orc_sim *s, int axis, int nslab, const double *edges, double *out);

#endif

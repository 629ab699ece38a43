/*
 * fd3d_oracle.c -- plain, slow FP64 CPU reference of the time-stepped 3D
 * elastic velocity-stress staggered-grid finite-difference scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or table with the HIP library; every rule is written out again here from
 * the paper (arXiv 2112.15071) and the readings listed beside each function.
 *
 * Paper passages followed:
 *   Sec. 2.1, Eq.(1)   rho dv/dt = div(sigma) + f
 *   Sec. 2.1, Eq.(2)   dsigma/dt = C : (1/2)(grad v + grad v^T), isotropic C(lambda, mu)
 *   Sec. 2.1, Eq.(3)   symmetric stress tensor, six independent components
 *   Sec. 2.1.1         Graves staggered positions of the nine fields
 *   Sec. 2.1.2, Eq.(4) fourth-order staggered first derivative (read as divided by the
 *                      spacing of its axis; Table 5 uses different cell sizes per axis)
 *   Sec. 2.2           one copy of each field, updated in place; velocity pass, then stress pass
 *   Sec. 2.2.1         effective rho, lambda, mu at staggered points by trilinear
 *                      interpolation of node values (= arithmetic means at half offsets)
 *   Sec. 2.4           receivers sampled by trilinear interpolation every step
 *   Sec. 2.5           damping factor near the edges (read as the Cerjan profile) and a
 *                      free top surface with a second-order z difference next to it
 *                      (read as stress imaging, see oracle_forward)
 *
 * Discrete conventions (identical readings are used by the GPU path, written
 * independently there):
 *   - nodes (i,j,k), x fastest: idx = i + nx*(j + ny*k); z points down, k = 0 is the top.
 *   - a component staggered along an axis holds n-1 active samples there (slot n-1 is
 *     pinned to zero); every sample outside the active range reads as zero.
 *   - D+ f[i] = (c1 (f[i+1]-f[i]) + c2 (f[i+2]-f[i-1])) / h_a  (integer -> half)
 *     D- g[i] = (c1 (g[i]-g[i-1]) + c2 (g[i+1]-g[i-2])) / h_a  (half -> integer)
 *     with h_a the spacing of the derivative's axis a
 *     c1 = 9/8, c2 = -1/24.
 *
 * Optional periodic axes exist for the dispersion pins only; the GPU path has none.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NF 9
enum { VX = 0, VY, VZ, SXX, SYY, SZZ, SXY, SXZ, SYZ };

/* Staggering per component (1 = half offset along that axis), Sec. 2.1.1. */
static const int STAG[NF][3] = {
    {1, 0, 0}, /* vx  at (x+1/2, y, z)       */
    {0, 1, 0}, /* vy  at (x, y+1/2, z)       */
    {0, 0, 1}, /* vz  at (x, y, z+1/2)       */
    {0, 0, 0}, /* sxx at (x, y, z)           */
    {0, 0, 0}, /* syy                        */
    {0, 0, 0}, /* szz                        */
    {1, 1, 0}, /* sxy at (x+1/2, y+1/2, z)   */
    {1, 0, 1}, /* sxz at (x+1/2, y, z+1/2)   */
    {0, 1, 1}, /* syz at (x, y+1/2, z+1/2)   */
};

/* Eq.(4) coefficients. */
static const double C1 = 9.0 / 8.0;
static const double C2 = -1.0 / 24.0;

typedef struct {
    int n[3];          /* nx, ny, nz */
    double h[3];       /* grid spacing per axis (m): dx, dy, dz */
    double dt;         /* time step (s) */
    int nt;            /* number of steps */
    int periodic[3];   /* oracle-only periodic axes */
    int free_surface;  /* stress-imaging free surface at k = 0 */
    int vacuum_top;    /* > 0: vacuum formulation, first solid node plane (the model
                          holds lam = mu = 0 above it); 0: off */
    const int *vacuum_map; /* optional [ny][nx]: first solid plane of each column
                              (topography); NULL: vacuum_top everywhere */
    int sponge[6];     /* damping width in cells: x-, x+, y-, y+, z- (top), z+ */
    double alpha;      /* Cerjan coefficient; <= 0 selects 0.3 / width per face */
    int coarse[3];     /* all > 0: the medium arrays hold a coarse node grid (mx, my, mz)
                          spanning the same box, and every medium value is a trilinear
                          sample of it at the value's own position (see coarse_at); all
                          0: the medium arrays are given at the simulation nodes */
} oracle_cfg;

typedef struct {
    double pos[3];     /* grid units (node spacing 1) */
    double moment[6];  /* Mxx Myy Mzz Mxy Mxz Myz, N m */
    double force[3];   /* Fx Fy Fz, N */
} oracle_src;

typedef struct {
    const oracle_cfg *c;
    const double *lam, *mu, *rho;
    double *prof[3][2];  /* damping profile per axis at integer [0] and half [1] positions */
} ctx_t;

static long nodes(const oracle_cfg *c) { return (long)c->n[0] * c->n[1] * c->n[2]; }
static long lin(const oracle_cfg *c, long i, long j, long k) { return i + (long)c->n[0] * (j + (long)c->n[1] * k); }

/* Map an index along one axis to storage; 0 when the sample is outside the active range. */
static int map_axis(const oracle_cfg *c, int axis, int stag, long i, long *out)
{
    int n = c->n[axis];
    if (c->periodic[axis]) {
        long m = i % n;
        if (m < 0) m += n;
        *out = m;
        return 1;
    }
    if (i < 0 || i > n - 1 - stag) return 0;
    *out = i;
    return 1;
}

static int active(const oracle_cfg *c, int comp, long i, long j, long k)
{
    long a = 0, b = 0, d = 0;
    return map_axis(c, 0, STAG[comp][0], i, &a) && map_axis(c, 1, STAG[comp][1], j, &b) &&
           map_axis(c, 2, STAG[comp][2], k, &d);
}

/* Value of a field sample; zero outside the active range (Sec. 2.2.2 replaced by a zero halo). */
static double get(const oracle_cfg *c, const double *f, int comp, long i, long j, long k)
{
    long a = 0, b = 0, d = 0;
    if (!map_axis(c, 0, STAG[comp][0], i, &a) || !map_axis(c, 1, STAG[comp][1], j, &b) ||
        !map_axis(c, 2, STAG[comp][2], k, &d))
        return 0.0;
    return f[a + (long)c->n[0] * (b + (long)c->n[1] * d)];
}

/* Stress read used by the velocity pass.  With the free surface, stresses above
 * k = 0 are odd images: szz(-m) = -szz(m); sxz, syz at z = -(m+1/2) mirror z = m+1/2. */
static double sget(const oracle_cfg *c, double *const *F, int comp, long i, long j, long k)
{
    if (c->free_surface && k < 0) {
        if (comp == SZZ) return -get(c, F[SZZ], SZZ, i, j, -k);
        if (comp == SXZ || comp == SYZ) return -get(c, F[comp], comp, i, j, -1 - k);
        return 0.0;
    }
    return get(c, F[comp], comp, i, j, k);
}

/* Vacuum formulation (Sec. 2.5): the z derivatives near the surface plane ks take the
 * second-order difference.  Reading: every z derivative whose result lies within one cell
 * of the surface, |z - ks| <= 1 -- half points ks - 1/2, ks + 1/2 (D+ from k = ks - 1, ks)
 * and integer points ks - 1, ks, ks + 1 (D-). */
/* Surface plane seen by a sample of component comp in column (i, j).  With topography
 * (a plane per node column) a sample between node columns -- at a half position in x or
 * y -- takes the deepest plane of the columns beside it (mirror-symmetric). */
static long surface_of(const oracle_cfg *c, int comp, long i, long j)
{
    if (!c->vacuum_map) return c->vacuum_top;
    long ks = 0;
    for (long a = 0; a <= STAG[comp][0]; ++a)
        for (long b = 0; b <= STAG[comp][1]; ++b) {
            long ii = i + a < c->n[0] ? i + a : c->n[0] - 1, jj = j + b < c->n[1] ? j + b : c->n[1] - 1;
            long v = c->vacuum_map[ii + (long)c->n[0] * jj];
            if (v > ks) ks = v;
        }
    return ks;
}

static int o2_plus(const oracle_cfg *c, int comp, int axis, long i, long j, long k)
{
    if (axis != 2 || c->vacuum_top <= 0) return 0;
    long ks = surface_of(c, comp, i, j);
    return k == ks - 1 || k == ks;
}

static int o2_minus(const oracle_cfg *c, int comp, int axis, long i, long j, long k)
{
    if (axis != 2 || c->vacuum_top <= 0) return 0;
    long ks = surface_of(c, comp, i, j);
    return k >= ks - 1 && k <= ks + 1;
}

/* Eq.(4), integer samples -> half point (slot i is position i+1/2 along the axis). */
static double dplus_s(const oracle_cfg *c, double *const *F, int comp, int axis, long i, long j, long k)
{
    long e0 = axis == 0, e1 = axis == 1, e2 = axis == 2;
    double f0 = sget(c, F, comp, i, j, k);
    double fp1 = sget(c, F, comp, i + e0, j + e1, k + e2);
    double fp2 = sget(c, F, comp, i + 2 * e0, j + 2 * e1, k + 2 * e2);
    double fm1 = sget(c, F, comp, i - e0, j - e1, k - e2);
    if (o2_plus(c, comp, axis, i, j, k)) return (fp1 - f0) / c->h[axis];
    return (C1 * (fp1 - f0) + C2 * (fp2 - fm1)) / c->h[axis];
}

/* Eq.(4), half samples -> integer point i. */
static double dminus_s(const oracle_cfg *c, double *const *F, int comp, int axis, long i, long j, long k)
{
    long e0 = axis == 0, e1 = axis == 1, e2 = axis == 2;
    double g0 = sget(c, F, comp, i, j, k);
    double gm1 = sget(c, F, comp, i - e0, j - e1, k - e2);
    double gp1 = sget(c, F, comp, i + e0, j + e1, k + e2);
    double gm2 = sget(c, F, comp, i - 2 * e0, j - 2 * e1, k - 2 * e2);
    if (o2_minus(c, comp, axis, i, j, k)) return (g0 - gm1) / c->h[axis];
    return (C1 * (g0 - gm1) + C2 * (gp1 - gm2)) / c->h[axis];
}

/* Same operators on velocity-like fields (no images; never read above the surface). */
static double dplus_v(const oracle_cfg *c, const double *f, int comp, int axis, long i, long j, long k)
{
    long e0 = axis == 0, e1 = axis == 1, e2 = axis == 2;
    double f0 = get(c, f, comp, i, j, k);
    double fp1 = get(c, f, comp, i + e0, j + e1, k + e2);
    double fp2 = get(c, f, comp, i + 2 * e0, j + 2 * e1, k + 2 * e2);
    double fm1 = get(c, f, comp, i - e0, j - e1, k - e2);
    if (o2_plus(c, comp, axis, i, j, k)) return (fp1 - f0) / c->h[axis];
    return (C1 * (fp1 - f0) + C2 * (fp2 - fm1)) / c->h[axis];
}

static double dminus_v(const oracle_cfg *c, const double *f, int comp, int axis, long i, long j, long k)
{
    long e0 = axis == 0, e1 = axis == 1, e2 = axis == 2;
    double g0 = get(c, f, comp, i, j, k);
    double gm1 = get(c, f, comp, i - e0, j - e1, k - e2);
    double gp1 = get(c, f, comp, i + e0, j + e1, k + e2);
    double gm2 = get(c, f, comp, i - 2 * e0, j - 2 * e1, k - 2 * e2);
    if (o2_minus(c, comp, axis, i, j, k)) return (g0 - gm1) / c->h[axis];
    return (C1 * (g0 - gm1) + C2 * (gp1 - gm2)) / c->h[axis];
}

/* Coarse medium (Sec. 2.2.1: the medium textures may be smaller than the simulation grid,
 * every read being a trilinear sample).  Reading: both grids span the same box corner node
 * to corner node, so simulation coordinate x (grid units, integer or half-integer) sits at
 * coarse coordinate X = x (m - 1) / (n - 1) per axis (an axis of m = 1 is constant); the
 * value is the trilinear interpolation of the eight coarse nodes around X -- the texture
 * read at the sample's own position, with no further averaging. */
static double coarse_at(const oracle_cfg *c, const double *m, double x, double y, double z)
{
    const double q[3] = {x, y, z};
    long lo[3], hi[3];
    double f[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int cm = c->coarse[ax], n = c->n[ax];
        double X = (cm > 1) ? q[ax] * (double)(cm - 1) / (double)(n - 1) : 0.0;
        if (X < 0.0) X = 0.0;
        if (X > cm - 1) X = cm - 1;
        long b = (long)floor(X);
        if (b > cm - 2) b = cm - 2;
        if (b < 0) b = 0;
        lo[ax] = b;
        hi[ax] = cm > 1 ? b + 1 : b;
        f[ax] = cm > 1 ? X - (double)b : 0.0;
    }
    double v = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                const long i = dx ? hi[0] : lo[0], j = dy ? hi[1] : lo[1], k = dz ? hi[2] : lo[2];
                v += w * m[i + (long)c->coarse[0] * (j + (long)c->coarse[1] * k)];
            }
    return v;
}

static int is_coarse(const oracle_cfg *c) { return c->coarse[0] > 0; }

/* Model value at a node (wrapping on periodic axes). */
static double node(const oracle_cfg *c, const double *m, long i, long j, long k)
{
    if (is_coarse(c)) return coarse_at(c, m, (double)i, (double)j, (double)k);
    long a = 0, b = 0, d = 0;
    map_axis(c, 0, 0, i, &a);
    map_axis(c, 1, 0, j, &b);
    map_axis(c, 2, 0, k, &d);
    return m[a + (long)c->n[0] * (b + (long)c->n[1] * d)];
}

/* Sec. 2.2.1: density at the velocity point of component comp (mean of the two nodes). */
static double rho_eff(const ctx_t *x, int comp, long i, long j, long k)
{
    long e0 = comp == VX, e1 = comp == VY, e2 = comp == VZ;
    if (is_coarse(x->c)) return coarse_at(x->c, x->rho, i + 0.5 * e0, j + 0.5 * e1, k + 0.5 * e2);
    return (node(x->c, x->rho, i, j, k) + node(x->c, x->rho, i + e0, j + e1, k + e2)) / 2.0;
}

/* Sec. 2.2.1: shear modulus at a shear-stress point (mean of the four nodes around it). */
static double mu_eff(const ctx_t *x, int comp, long i, long j, long k)
{
    long a0 = STAG[comp][0], a1 = STAG[comp][1], a2 = STAG[comp][2];
    if (is_coarse(x->c)) return coarse_at(x->c, x->mu, i + 0.5 * a0, j + 0.5 * a1, k + 0.5 * a2);
    /* the two staggered axes of this component */
    long u[3] = {0, 0, 0}, w[3] = {0, 0, 0};
    int first = 1;
    long s[3] = {a0, a1, a2};
    for (int ax = 0; ax < 3; ++ax) {
        if (!s[ax]) continue;
        if (first) { u[ax] = 1; first = 0; }
        else w[ax] = 1;
    }
    double m00 = node(x->c, x->mu, i, j, k);
    double m10 = node(x->c, x->mu, i + u[0], j + u[1], k + u[2]);
    double m01 = node(x->c, x->mu, i + w[0], j + w[1], k + w[2]);
    double m11 = node(x->c, x->mu, i + u[0] + w[0], j + u[1] + w[1], k + u[2] + w[2]);
    return ((m00 + m10) + (m01 + m11)) / 4.0;
}

/* Sec. 2.5 read as Cerjan damping: g(d) = exp(-(a (nb - d))^2) for d < nb, with d the
 * distance (cells) from the face measured at the sample's own coordinate. */
static double face_factor(double d, int nb, double alpha)
{
    if (nb <= 0 || d >= nb) return 1.0;
    double a = alpha > 0.0 ? alpha : 0.3 / nb;
    double t = a * (nb - d);
    return exp(-t * t);
}

static void build_profiles(ctx_t *x)
{
    const oracle_cfg *c = x->c;
    for (int ax = 0; ax < 3; ++ax) {
        int n = c->n[ax];
        int lo = c->sponge[2 * ax], hi = c->sponge[2 * ax + 1];
        if (c->periodic[ax]) lo = hi = 0;
        if (ax == 2 && c->free_surface) lo = 0;
        for (int half = 0; half < 2; ++half) {
            double *p = (double *)malloc(sizeof(double) * n);
            for (int i = 0; i < n; ++i) {
                double pos = i + 0.5 * half;
                p[i] = face_factor(pos, lo, c->alpha) * face_factor((n - 1) - pos, hi, c->alpha);
            }
            x->prof[ax][half] = p;
        }
    }
}

static void free_profiles(ctx_t *x)
{
    for (int ax = 0; ax < 3; ++ax)
        for (int h = 0; h < 2; ++h) free(x->prof[ax][h]);
}

/* Damping factor G = gx gy gz at the sample (i,j,k) of component comp. */
static double damp(const ctx_t *x, int comp, long i, long j, long k)
{
    return x->prof[0][STAG[comp][0]][i] * x->prof[1][STAG[comp][1]][j] * x->prof[2][STAG[comp][2]][k];
}

/* Trilinear point operator (Sec. 2.4) on the component's own subgrid: the eight taps and
 * weights of point p (grid units) after removing the component's staggering offset. */
typedef struct { long i[8], j[8], k[8]; double w[8]; } taps_t;

static void point_taps(int comp, const double *p, taps_t *t)
{
    double q[3];
    long b[3];
    double f[3];
    for (int ax = 0; ax < 3; ++ax) {
        q[ax] = p[ax] - 0.5 * STAG[comp][ax];
        b[ax] = (long)floor(q[ax]);
        f[ax] = q[ax] - (double)b[ax];
    }
    int m = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                t->i[m] = b[0] + dx;
                t->j[m] = b[1] + dy;
                t->k[m] = b[2] + dz;
                t->w[m] = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                ++m;
            }
}

static double sample(const oracle_cfg *c, const double *f, int comp, const double *p)
{
    taps_t t;
    point_taps(comp, p, &t);
    double s = 0.0;
    for (int m = 0; m < 8; ++m) s += t.w[m] * get(c, f, comp, t.i[m], t.j[m], t.k[m]);
    return s;
}

/* Adds amp * w to every active tap of a point operator (transpose of sample). */
static void inject(const oracle_cfg *c, double *f, int comp, const double *p, const double *amp_per_tap)
{
    taps_t t;
    point_taps(comp, p, &t);
    for (int m = 0; m < 8; ++m) {
        if (!active(c, comp, t.i[m], t.j[m], t.k[m])) continue;
        long a = 0, b = 0, d = 0;
        map_axis(c, 0, STAG[comp][0], t.i[m], &a);
        map_axis(c, 1, STAG[comp][1], t.j[m], &b);
        map_axis(c, 2, STAG[comp][2], t.k[m], &d);
        f[lin(c, a, b, d)] += t.w[m] * amp_per_tap[m];
    }
}

/* div(sigma) at the velocity sample of component comp, Eq.(1) with Eq.(4). */
static double div_sigma(const oracle_cfg *c, double *const *F, int comp, long i, long j, long k)
{
    if (comp == VX)
        return dplus_s(c, F, SXX, 0, i, j, k) + dminus_s(c, F, SXY, 1, i, j, k) + dminus_s(c, F, SXZ, 2, i, j, k);
    if (comp == VY)
        return dminus_s(c, F, SXY, 0, i, j, k) + dplus_s(c, F, SYY, 1, i, j, k) + dminus_s(c, F, SYZ, 2, i, j, k);
    return dminus_s(c, F, SXZ, 0, i, j, k) + dminus_s(c, F, SYZ, 1, i, j, k) + dplus_s(c, F, SZZ, 2, i, j, k);
}

/* Strain rates at a normal-stress node: exx, eyy, ezz (Eq.(2) with Eq.(4)), with the
 * free-surface rules at k = 0 (ezz from szz = 0) and k = 1 (second-order ezz). */
static void normal_strain(const ctx_t *x, const double *const *V, long i, long j, long k, double e[3])
{
    const oracle_cfg *c = x->c;
    e[0] = dminus_v(c, V[VX], VX, 0, i, j, k);
    e[1] = dminus_v(c, V[VY], VY, 1, i, j, k);
    if (c->free_surface && k == 0) {
        double l = node(c, x->lam, i, j, k), m = node(c, x->mu, i, j, k);
        e[2] = -l / (l + 2.0 * m) * (e[0] + e[1]);
    } else if (c->free_surface && k == 1) {
        e[2] = (get(c, V[VZ], VZ, i, j, 1) - get(c, V[VZ], VZ, i, j, 0)) / c->h[2];
    } else {
        e[2] = dminus_v(c, V[VZ], VZ, 2, i, j, k);
    }
}

/* Engineering shear strain rate at a shear-stress sample (d_a v_b + d_b v_a). */
static double shear_strain(const ctx_t *x, const double *const *V, int comp, long i, long j, long k)
{
    const oracle_cfg *c = x->c;
    if (comp == SXY) return dplus_v(c, V[VX], VX, 1, i, j, k) + dplus_v(c, V[VY], VY, 0, i, j, k);
    if (comp == SXZ) {
        double dzvx = (c->free_surface && k == 0)
                          ? (get(c, V[VX], VX, i, j, 1) - get(c, V[VX], VX, i, j, 0)) / c->h[2]
                          : dplus_v(c, V[VX], VX, 2, i, j, k);
        return dzvx + dplus_v(c, V[VZ], VZ, 0, i, j, k);
    }
    double dzvy = (c->free_surface && k == 0)
                      ? (get(c, V[VY], VY, i, j, 1) - get(c, V[VY], VY, i, j, 0)) / c->h[2]
                      : dplus_v(c, V[VY], VY, 2, i, j, k);
    return dzvy + dplus_v(c, V[VZ], VZ, 1, i, j, k);
}

/* ---------------- one time step ---------------- */

/* Volume of one cell, dx dy dz (the point sources inject per unit volume). */
static double cell_volume(const oracle_cfg *c) { return c->h[0] * c->h[1] * c->h[2]; }

/* (V) velocity pass: v <- G (v + dt b div(sigma) + dt b w F s / (dx dy dz)). */
static void velocity_pass(const ctx_t *x, double *const *F, const oracle_src *src, double s)
{
    const oracle_cfg *c = x->c;
    long nx = c->n[0], ny = c->n[1], nz = c->n[2];
    for (int comp = VX; comp <= VZ; ++comp) {
#pragma omp parallel for schedule(static)
        for (long k = 0; k < nz; ++k)
            for (long j = 0; j < ny; ++j)
                for (long i = 0; i < nx; ++i) {
                    if (!active(c, comp, i, j, k)) continue;
                    double b = 1.0 / rho_eff(x, comp, i, j, k);
                    F[comp][lin(c, i, j, k)] += c->dt * b * div_sigma(c, F, comp, i, j, k);
                }
        if (src && src->force[comp] != 0.0) {
            taps_t t;
            point_taps(comp, src->pos, &t);
            double amp[8];
            for (int m = 0; m < 8; ++m) {
                double b = active(c, comp, t.i[m], t.j[m], t.k[m]) ? 1.0 / rho_eff(x, comp, t.i[m], t.j[m], t.k[m]) : 0.0;
                amp[m] = c->dt * b * src->force[comp] * s / cell_volume(c);
            }
            inject(c, F[comp], comp, src->pos, amp);
        }
#pragma omp parallel for schedule(static)
        for (long k = 0; k < nz; ++k)
            for (long j = 0; j < ny; ++j)
                for (long i = 0; i < nx; ++i) F[comp][lin(c, i, j, k)] *= damp(x, comp, i, j, k);
    }
}

/* (S) stress pass: sigma <- G (sigma + dt C:eps(v) - dt w M s / (dx dy dz)); szz(k=0) = 0 with
 * the free surface. Reads only velocities, so all six components update in place. */
static void stress_pass(const ctx_t *x, double *const *F, const oracle_src *src, double s)
{
    const oracle_cfg *c = x->c;
    long nx = c->n[0], ny = c->n[1], nz = c->n[2];
    const double *const *V = (const double *const *)F;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = lin(c, i, j, k);
                double e[3];
                normal_strain(x, V, i, j, k, e);
                double l = node(c, x->lam, i, j, k), m = node(c, x->mu, i, j, k);
                double tr = e[0] + e[1] + e[2];
                F[SXX][p] += c->dt * (l * tr + 2.0 * m * e[0]);
                F[SYY][p] += c->dt * (l * tr + 2.0 * m * e[1]);
                F[SZZ][p] += c->dt * (l * tr + 2.0 * m * e[2]);
                for (int comp = SXY; comp <= SYZ; ++comp) {
                    if (!active(c, comp, i, j, k)) continue;
                    F[comp][p] += c->dt * mu_eff(x, comp, i, j, k) * shear_strain(x, V, comp, i, j, k);
                }
            }
    if (src) {
        for (int q = 0; q < 6; ++q) {
            int comp = SXX + q;
            if (src->moment[q] == 0.0) continue;
            double amp[8];
            for (int m = 0; m < 8; ++m) amp[m] = -c->dt * src->moment[q] * s / cell_volume(c);
            inject(c, F[comp], comp, src->pos, amp);
        }
    }
    for (int comp = SXX; comp <= SYZ; ++comp) {
#pragma omp parallel for schedule(static)
        for (long k = 0; k < nz; ++k)
            for (long j = 0; j < ny; ++j)
                for (long i = 0; i < nx; ++i) F[comp][lin(c, i, j, k)] *= damp(x, comp, i, j, k);
    }
    if (c->free_surface) {
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) F[SZZ][lin(c, i, j, 0)] = 0.0;
    }
}

static int check_cfg(const oracle_cfg *c)
{
    for (int a = 0; a < 3; ++a)
        if (c->n[a] < 2) return -1;
    if (!(c->h[0] > 0.0) || !(c->h[1] > 0.0) || !(c->h[2] > 0.0) || !(c->dt > 0.0) || c->nt < 0) return -1;
    if (c->free_surface && c->periodic[2]) return -1;
    if (c->vacuum_top < 0 || c->vacuum_top >= c->n[2] || (c->vacuum_top > 0 && (c->free_surface || c->periodic[2])))
        return -1;
    if (c->coarse[0] || c->coarse[1] || c->coarse[2]) {
        for (int a = 0; a < 3; ++a)
            if (c->coarse[a] < 1 || c->periodic[a]) return -1;
    }
    if (c->vacuum_map) {
        if (c->vacuum_top <= 0) return -1;
        for (long q = 0; q < (long)c->n[0] * c->n[1]; ++q)
            if (c->vacuum_map[q] < 1 || c->vacuum_map[q] >= c->n[2]) return -1;
    }
    return 0;
}

/*
 * Forward simulation.  state: 9 arrays of N doubles, packed [9][N] in the order
 * vx vy vz sxx syy szz sxy sxz syz.  If use_state_in is 0 the state starts at zero
 * (v^{-1/2} = 0, sigma^0 = 0); otherwise it starts from the given arrays.  On return
 * it holds v^{nt-1/2} and sigma^{nt}.  traces: [nrec][3][nt], v^{n+1/2} sampled after
 * the velocity pass of step n.  wavelet[n] is used by both source kinds at step n.
 */
int oracle_forward(const oracle_cfg *cfg, const double *lam, const double *mu, const double *rho,
                   const oracle_src *src, const double *wavelet, int nrec, const double *rec_pos,
                   double *traces, double *state, int use_state_in)
{
    if (check_cfg(cfg)) return -1;
    ctx_t x = {cfg, lam, mu, rho, {{0}}};
    build_profiles(&x);
    long N = nodes(cfg);
    double *F[NF];
    for (int f = 0; f < NF; ++f) F[f] = state + (long)f * N;
    if (!use_state_in) memset(state, 0, sizeof(double) * NF * N);
    for (int n = 0; n < cfg->nt; ++n) {
        double s = wavelet ? wavelet[n] : 0.0;
        velocity_pass(&x, F, src, s);
        for (int r = 0; r < nrec; ++r)
            for (int cc = 0; cc < 3; ++cc)
                traces[((long)r * 3 + cc) * cfg->nt + n] = sample(cfg, F[VX + cc], VX + cc, rec_pos + 3 * r);
        stress_pass(&x, F, src, s);
    }
    free_profiles(&x);
    return 0;
}

/* ---------------- tangent-linear (Born) forward ---------------- */

/*
 * Derivative of oracle_forward's traces with respect to the node arrays lam, mu, rho
 * along (dlam, dmu, drho), taken step by step through the same three steps (velocity
 * pass, sampling, stress pass).  With b = 1/rho_eff and C(lam, mu) as in the forward:
 *   velocity:  dv     <- G (dv + dt b D_S dsigma + dt db (D_S sigma + w F s / V))
 *   sampling:  dd[n]   = W dv^{n+1/2}
 *   stress:    dsigma <- G (dsigma + dt C E(dv) + dt dC E(v))
 * where db = -b^2 drho_eff (drho_eff the two-node mean of drho), dC the same matrix as
 * C built from dlam, dmu (dmu at shear points the four-node mean), and v, sigma the
 * background at the same point of the step.  The perturbation starts at zero.  No free
 * surface.  dtraces: [nrec][3][nt]; traces (may be NULL) receives the background.
 */
int oracle_born(const oracle_cfg *cfg, const double *lam, const double *mu, const double *rho,
                const double *dlam, const double *dmu, const double *drho, const oracle_src *src,
                const double *wavelet, int nrec, const double *rec_pos, double *traces, double *dtraces)
{
    if (check_cfg(cfg) || cfg->free_surface || cfg->vacuum_top || is_coarse(cfg)) return -1;
    const oracle_cfg *c = cfg;
    ctx_t x = {cfg, lam, mu, rho, {{0}}};
    ctx_t dx = {cfg, dlam, dmu, drho, {{0}}};  /* perturbation arrays, for the same means */
    build_profiles(&x);
    long N = nodes(c), nx = c->n[0], ny = c->n[1], nz = c->n[2];
    double *state = (double *)calloc((size_t)NF * N, sizeof(double));
    double *dstate = (double *)calloc((size_t)NF * N, sizeof(double));
    if (!state || !dstate) { free(state); free(dstate); free_profiles(&x); return -2; }
    double *F[NF], *D[NF];
    for (int f = 0; f < NF; ++f) { F[f] = state + (long)f * N; D[f] = dstate + (long)f * N; }
    for (int n = 0; n < c->nt; ++n) {
        double s = wavelet ? wavelet[n] : 0.0;
        /* velocity: the buoyancy perturbation acting on the background stress and force */
        for (int comp = VX; comp <= VZ; ++comp) {
#pragma omp parallel for schedule(static)
            for (long k = 0; k < nz; ++k)
                for (long j = 0; j < ny; ++j)
                    for (long i = 0; i < nx; ++i) {
                        if (!active(c, comp, i, j, k)) continue;
                        double b = 1.0 / rho_eff(&x, comp, i, j, k);
                        double db = -b * b * rho_eff(&dx, comp, i, j, k);
                        D[comp][lin(c, i, j, k)] += c->dt * db * div_sigma(c, F, comp, i, j, k);
                    }
            if (src && src->force[comp] != 0.0) {
                taps_t t;
                point_taps(comp, src->pos, &t);
                double amp[8];
                for (int m = 0; m < 8; ++m) {
                    double db = 0.0;
                    if (active(c, comp, t.i[m], t.j[m], t.k[m])) {
                        double b = 1.0 / rho_eff(&x, comp, t.i[m], t.j[m], t.k[m]);
                        db = -b * b * rho_eff(&dx, comp, t.i[m], t.j[m], t.k[m]);
                    }
                    amp[m] = c->dt * db * src->force[comp] * s / cell_volume(c);
                }
                inject(c, D[comp], comp, src->pos, amp);
            }
        }
        velocity_pass(&x, D, NULL, 0.0); /* dv <- G (dv + ... + dt b D_S dsigma) */
        velocity_pass(&x, F, src, s);
        for (int r = 0; r < nrec; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                long o = ((long)r * 3 + cc) * c->nt + n;
                dtraces[o] = sample(c, D[VX + cc], VX + cc, rec_pos + 3 * r);
                if (traces) traces[o] = sample(c, F[VX + cc], VX + cc, rec_pos + 3 * r);
            }
        /* stress: the stiffness perturbation acting on the new background velocity */
        {
            const double *const *V = (const double *const *)F;
#pragma omp parallel for schedule(static)
            for (long k = 0; k < nz; ++k)
                for (long j = 0; j < ny; ++j)
                    for (long i = 0; i < nx; ++i) {
                        long p = lin(c, i, j, k);
                        double e[3];
                        normal_strain(&x, V, i, j, k, e);
                        double l = node(c, dlam, i, j, k), m = node(c, dmu, i, j, k);
                        double tr = e[0] + e[1] + e[2];
                        D[SXX][p] += c->dt * (l * tr + 2.0 * m * e[0]);
                        D[SYY][p] += c->dt * (l * tr + 2.0 * m * e[1]);
                        D[SZZ][p] += c->dt * (l * tr + 2.0 * m * e[2]);
                        for (int comp = SXY; comp <= SYZ; ++comp) {
                            if (!active(c, comp, i, j, k)) continue;
                            D[comp][p] += c->dt * mu_eff(&dx, comp, i, j, k) * shear_strain(&x, V, comp, i, j, k);
                        }
                    }
        }
        stress_pass(&x, D, NULL, 0.0); /* dsigma <- G (dsigma + ... + dt C E dv) */
        stress_pass(&x, F, src, s);
    }
    free(state);
    free(dstate);
    free_profiles(&x);
    return 0;
}

/* ---------------- discrete adjoint (store-all, small grids) ---------------- */

/*
 * Gradient of J = 1/2 sum (d - d_obs)^2 with respect to the node arrays lam, mu, rho,
 * given residual = dJ/dd [nrec][3][nt].  The adjoint is the exact transpose of the
 * steps of oracle_forward (velocity pass, sampling, stress pass), taken in reverse
 * order, with every forward state stored.  No free surface.  The derivative
 * operators satisfy D- = -(D+)^T under the zero-halo rules, which the adjoint uses
 * to apply the transposed passes.
 *
 * If adj_state is not NULL it receives the adjoint of the initial state
 * [9][N] (adjoint of v^{-1/2} and sigma^0), for the dot-product pins.
 */
int oracle_gradient(const oracle_cfg *cfg, const double *lam, const double *mu, const double *rho,
                    const oracle_src *src, const double *wavelet, int nrec, const double *rec_pos,
                    const double *residual, const double *state0, double *g_lam, double *g_mu,
                    double *g_rho, double *adj_state)
{
    if (check_cfg(cfg) || cfg->free_surface || cfg->vacuum_top || is_coarse(cfg)) return -1;
    const oracle_cfg *c = cfg;
    ctx_t x = {cfg, lam, mu, rho, {{0}}};
    build_profiles(&x);
    long N = nodes(c), nx = c->n[0], ny = c->n[1], nz = c->n[2];
    int nt = c->nt;
    double h3 = cell_volume(c);

    /* forward, storing sigma^n (before step n) and v^{n+1/2} (after the velocity pass) */
    double *Sst = (double *)malloc(sizeof(double) * 6 * N * (size_t)nt);
    double *Vst = (double *)malloc(sizeof(double) * 3 * N * (size_t)nt);
    double *state = (double *)calloc((size_t)NF * N, sizeof(double));
    if (!Sst || !Vst || !state) { free(Sst); free(Vst); free(state); free_profiles(&x); return -2; }
    if (state0) memcpy(state, state0, sizeof(double) * NF * N);
    double *F[NF];
    for (int f = 0; f < NF; ++f) F[f] = state + (long)f * N;
    for (int n = 0; n < nt; ++n) {
        double s = wavelet ? wavelet[n] : 0.0;
        memcpy(Sst + (size_t)n * 6 * N, F[SXX], sizeof(double) * 6 * N);
        velocity_pass(&x, F, src, s);
        memcpy(Vst + (size_t)n * 3 * N, F[VX], sizeof(double) * 3 * N);
        stress_pass(&x, F, src, s);
    }

    /* adjoint variables and gradients at staggered points */
    double *A = (double *)calloc((size_t)NF * N, sizeof(double)); /* vbar, sbar */
    double *X = (double *)calloc((size_t)6 * N, sizeof(double));  /* C applied to T */
    double *Y = (double *)calloc((size_t)3 * N, sizeof(double));  /* b applied to U */
    double *gl = (double *)calloc(N, sizeof(double));
    double *gmn = (double *)calloc(N, sizeof(double));
    double *gms = (double *)calloc((size_t)3 * N, sizeof(double)); /* mu_xy, mu_xz, mu_yz */
    double *gb = (double *)calloc((size_t)3 * N, sizeof(double));  /* b_x, b_y, b_z */
    double *Ab[NF], *Xb[NF];
    for (int f = 0; f < NF; ++f) Ab[f] = A + (long)f * N;
    for (int f = 0; f < 6; ++f) Xb[SXX + f] = X + (long)f * N;
    for (int f = 0; f < 3; ++f) Xb[f] = Y + (long)f * N;

    for (int n = nt - 1; n >= 0; --n) {
        double s = wavelet ? wavelet[n] : 0.0;
        double *Vn[3] = {Vst + (size_t)n * 3 * N, Vst + (size_t)n * 3 * N + N, Vst + (size_t)n * 3 * N + 2 * N};
        double *Sn[NF];
        for (int f = 0; f < 6; ++f) Sn[SXX + f] = Sst + (size_t)n * 6 * N + (long)f * N;
        Sn[VX] = Sn[VY] = Sn[VZ] = NULL;

        /* adjoint of the stress pass: T = G_s sbar; gradients of C; vbar -= dt D_S(C T); sbar = T */
        for (int comp = SXX; comp <= SYZ; ++comp)
#pragma omp parallel for schedule(static)
            for (long k = 0; k < nz; ++k)
                for (long j = 0; j < ny; ++j)
                    for (long i = 0; i < nx; ++i) Ab[comp][lin(c, i, j, k)] *= damp(&x, comp, i, j, k);
        {
            const double *Vc[3] = {Vn[0], Vn[1], Vn[2]};
#pragma omp parallel for schedule(static)
            for (long k = 0; k < nz; ++k)
                for (long j = 0; j < ny; ++j)
                    for (long i = 0; i < nx; ++i) {
                        long p = lin(c, i, j, k);
                        double e[3];
                        normal_strain(&x, Vc, i, j, k, e);
                        double l = node(c, lam, i, j, k), m = node(c, mu, i, j, k);
                        double txx = Ab[SXX][p], tyy = Ab[SYY][p], tzz = Ab[SZZ][p];
                        double trT = txx + tyy + tzz, tre = e[0] + e[1] + e[2];
                        gl[p] += c->dt * tre * trT;
                        gmn[p] += c->dt * 2.0 * (e[0] * txx + e[1] * tyy + e[2] * tzz);
                        Xb[SXX][p] = l * trT + 2.0 * m * txx;
                        Xb[SYY][p] = l * trT + 2.0 * m * tyy;
                        Xb[SZZ][p] = l * trT + 2.0 * m * tzz;
                        for (int comp = SXY; comp <= SYZ; ++comp) {
                            if (!active(c, comp, i, j, k)) { Xb[comp][p] = 0.0; continue; }
                            double t = Ab[comp][p];
                            gms[(long)(comp - SXY) * N + p] += c->dt * shear_strain(&x, Vc, comp, i, j, k) * t;
                            Xb[comp][p] = mu_eff(&x, comp, i, j, k) * t;
                        }
                    }
        }
        for (int comp = VX; comp <= VZ; ++comp)
#pragma omp parallel for schedule(static)
            for (long k = 0; k < nz; ++k)
                for (long j = 0; j < ny; ++j)
                    for (long i = 0; i < nx; ++i) {
                        if (!active(c, comp, i, j, k)) continue;
                        Ab[comp][lin(c, i, j, k)] -= c->dt * div_sigma(c, Xb, comp, i, j, k);
                    }

        /* adjoint of the sampling: vbar += W^T r^n */
        for (int r = 0; r < nrec; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                double rv = residual[((long)r * 3 + cc) * nt + n];
                double amp[8];
                for (int m = 0; m < 8; ++m) amp[m] = rv;
                inject(c, Ab[VX + cc], VX + cc, rec_pos + 3 * r, amp);
            }

        /* adjoint of the velocity pass: U = G_v vbar; g_b += dt (D_S sigma^n + w F s/(dx dy dz)) U;
         * sbar -= dt E(b U); vbar = U */
        for (int comp = VX; comp <= VZ; ++comp) {
#pragma omp parallel for schedule(static)
            for (long k = 0; k < nz; ++k)
                for (long j = 0; j < ny; ++j)
                    for (long i = 0; i < nx; ++i) {
                        long p = lin(c, i, j, k);
                        Ab[comp][p] *= damp(&x, comp, i, j, k);
                        if (!active(c, comp, i, j, k)) { Xb[comp][p] = 0.0; continue; }
                        double u = Ab[comp][p];
                        gb[(long)comp * N + p] += c->dt * div_sigma(c, Sn, comp, i, j, k) * u;
                        Xb[comp][p] = u / rho_eff(&x, comp, i, j, k);
                    }
            if (src && src->force[comp] != 0.0) {
                taps_t t;
                point_taps(comp, src->pos, &t);
                for (int m = 0; m < 8; ++m) {
                    if (!active(c, comp, t.i[m], t.j[m], t.k[m])) continue;
                    long p = lin(c, t.i[m], t.j[m], t.k[m]);
                    gb[(long)comp * N + p] += c->dt * t.w[m] * src->force[comp] * s / h3 * Ab[comp][p];
                }
            }
        }
        {
            const double *Yc[3] = {Xb[VX], Xb[VY], Xb[VZ]};
#pragma omp parallel for schedule(static)
            for (long k = 0; k < nz; ++k)
                for (long j = 0; j < ny; ++j)
                    for (long i = 0; i < nx; ++i) {
                        long p = lin(c, i, j, k);
                        double e[3];
                        normal_strain(&x, Yc, i, j, k, e);
                        Ab[SXX][p] -= c->dt * e[0];
                        Ab[SYY][p] -= c->dt * e[1];
                        Ab[SZZ][p] -= c->dt * e[2];
                        for (int comp = SXY; comp <= SYZ; ++comp) {
                            if (!active(c, comp, i, j, k)) continue;
                            Ab[comp][p] -= c->dt * shear_strain(&x, Yc, comp, i, j, k);
                        }
                    }
        }
    }

    /* chain rule to the node arrays (Sec. 2.2.1 averages) */
    for (long p = 0; p < N; ++p) { g_lam[p] = gl[p]; g_mu[p] = gmn[p]; g_rho[p] = 0.0; }
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = lin(c, i, j, k);
                for (int comp = SXY; comp <= SYZ; ++comp) {
                    if (!active(c, comp, i, j, k)) continue;
                    double g = gms[(long)(comp - SXY) * N + p] / 4.0;
                    long u0 = STAG[comp][0], u1 = STAG[comp][1], u2 = STAG[comp][2];
                    /* the four nodes of the mean: offsets over the two staggered axes */
                    for (long a = 0; a <= u0; ++a)
                        for (long b = 0; b <= u1; ++b)
                            for (long d = 0; d <= u2; ++d) {
                                long ii = 0, jj = 0, kk = 0;
                                map_axis(c, 0, 0, i + a, &ii);
                                map_axis(c, 1, 0, j + b, &jj);
                                map_axis(c, 2, 0, k + d, &kk);
                                g_mu[lin(c, ii, jj, kk)] += g;
                            }
                }
                for (int comp = VX; comp <= VZ; ++comp) {
                    if (!active(c, comp, i, j, k)) continue;
                    double re = rho_eff(&x, comp, i, j, k);
                    double g = -gb[(long)comp * N + p] / (re * re) / 2.0; /* db/drho_node = -b^2/2 */
                    long ii = 0, jj = 0, kk = 0;
                    g_rho[p] += g;
                    map_axis(c, 0, 0, i + (comp == VX), &ii);
                    map_axis(c, 1, 0, j + (comp == VY), &jj);
                    map_axis(c, 2, 0, k + (comp == VZ), &kk);
                    g_rho[lin(c, ii, jj, kk)] += g;
                }
            }
    if (adj_state) memcpy(adj_state, A, sizeof(double) * NF * N);

    free(Sst); free(Vst); free(state); free(A); free(X); free(Y);
    free(gl); free(gmn); free(gms); free(gb);
    free_profiles(&x);
    return 0;
}

/* Damping profiles as built above, exported for the pins: out[ax][half][n]. */
/* The medium values the scheme uses (Sec. 2.2.1), eight arrays [nz][ny][nx] into out:
 * rho at the vx, vy, vz samples, lambda and mu at the nodes, mu at the sxy, sxz, syz
 * samples; zero at inactive (pinned) samples.  Node means of node arrays, or trilinear
 * samples of a coarse grid (cfg->coarse). */
int oracle_medium(const oracle_cfg *cfg, const double *lam, const double *mu, const double *rho, double *out)
{
    if (check_cfg(cfg)) return -1;
    ctx_t x = {cfg, lam, mu, rho, {{0}}};
    long N = nodes(cfg);
    for (long k = 0; k < cfg->n[2]; ++k)
        for (long j = 0; j < cfg->n[1]; ++j)
            for (long i = 0; i < cfg->n[0]; ++i) {
                long p = lin(cfg, i, j, k);
                for (int comp = VX; comp <= VZ; ++comp)
                    out[(comp - VX) * N + p] = active(cfg, comp, i, j, k) ? rho_eff(&x, comp, i, j, k) : 0.0;
                out[3 * N + p] = node(cfg, lam, i, j, k);
                out[4 * N + p] = node(cfg, mu, i, j, k);
                for (int comp = SXY; comp <= SYZ; ++comp)
                    out[(5 + comp - SXY) * N + p] = active(cfg, comp, i, j, k) ? mu_eff(&x, comp, i, j, k) : 0.0;
            }
    return 0;
}

int oracle_profiles(const oracle_cfg *cfg, double *out)
{
    ctx_t x = {cfg, NULL, NULL, NULL, {{0}}};
    build_profiles(&x);
    long off = 0;
    for (int ax = 0; ax < 3; ++ax)
        for (int h = 0; h < 2; ++h) {
            memcpy(out + off, x.prof[ax][h], sizeof(double) * cfg->n[ax]);
            off += cfg->n[ax];
        }
    free_profiles(&x);
    return 0;
}

/* The staggered derivative operators of Eq.(4) on one 1D line, exported for the pins.
 * plus != 0: integer samples in[0..n-1] -> half points (slot n-1 pinned to 0);
 * plus == 0: half samples in[0..n-2] (in[n-1] ignored) -> integer points. */
int oracle_deriv1d(int n, double h, int plus, const double *in, double *out)
{
    oracle_cfg c;
    memset(&c, 0, sizeof c);
    c.n[0] = n; c.n[1] = 1; c.n[2] = 1; c.h[0] = c.h[1] = c.h[2] = h; c.dt = 1.0;
    for (long i = 0; i < n; ++i) {
        if (plus) out[i] = (i <= n - 2) ? dplus_v(&c, in, SXX, 0, i, 0, 0) : 0.0;
        else out[i] = dminus_v(&c, in, VX, 0, i, 0, 0);
    }
    return 0;
}

/* Thread control for the CPU-baseline timing (OpenMP over the outer z loop). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Oracle: plain, slow FP64 lattice-Boltzmann time stepper for the paper's
 * discrete velocity models with the diffuse Maxwell wall.
 *
 * TEST INFRASTRUCTURE. Only tests, the smoke check and the CPU-baseline leg of
 * the benchmark load this library. It shares no code, header or table with the
 * product library.
 *
 * Layout: array-of-structures, f[node * V + alpha], node = (k * ny + j) * nx + i.
 * The x direction is periodic; walls sit half a spacing outside the first and
 * last node in y (and in z for a duct), i.e. the half-way placement of
 * Section V. Separate passes: stream (with wall slots), moments, equilibrium,
 * force, collide.
 *
 * Equations followed (Section V, "Numerical method", unless noted):
 *   - equilibrium: tensor Hermite expansion to order N with coefficients
 *     rho u...u (Eqs. equi.hermite, equi.hermite.coef), Hermite tensors
 *     H_{i1..in}(xi) = prod_d He_{n_d}(xi_d) (the product form of Eq. defH);
 *   - body force: third-order Hermite expansion, Eq. nm.4, generalised
 *     equilibrium f^eq = f^(0) + tau F (Eq. nm.2);
 *   - explicit update on the modified populations (Eqs. nm.7, nm.8):
 *     fbar*(x) = fbar(x) - omega (fbar - f^eq), omega = dt / (tau + dt/2);
 *   - moments from fbar with the half-force shift (Eq. nm.10);
 *   - the second moment of the physical f entering nm.4 is recovered from
 *     fbar by inverting Eq. nm.7;
 *   - diffuse Maxwell wall (Eqs. nm.14, nm.15) on the unknown populations,
 *     transformed to fbar with the wall's own generalised equilibrium at
 *     u = 0: fbar = rho_eff * w * (1 - dt/2 g.xi). rho_eff per wall element
 *     is fixed by the discrete balance "mass emitted = mass absorbed" over the
 *     populations that cross the wall in one step (Eq. nm.15 counts them with
 *     the weight |n.xi|; on the lattice a population with |e_n| = m crosses
 *     from m rows). A wall element is the cell of the fluid node next to the
 *     crossing, on the face crossed first going outward from that node.
 *   - Maxwell's accommodation alpha < 1 (not treated in the paper, which
 *     takes the fully diffuse wall; channel walls normal to y only): the
 *     diffuse part re-emits alpha times the absorbed populations as above,
 *     and a fraction 1 - alpha is reflected specularly, i.e. with the wall
 *     normal velocity component reversed. The specular partner of the slot
 *     (x, alpha) is the population with the reflected velocity that leaves
 *     from the image of the virtual source x - e_alpha in the wall plane.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int dim;          /* 2 or 3 */
    int V;            /* number of velocities */
    int N;            /* Hermite order of the equilibrium */
    int nx, ny, nz;   /* nodes; nz = 1 in 2D */
    int walls_z;      /* 1: walls on the two z faces too (duct) */
    int pad_;
    const int *e;     /* V x 3 integer velocities, xi = c * e (e_z = 0 in 2D) */
    const double *w;  /* V weights */
    double c;         /* lattice speed */
    double tau;       /* relaxation time */
    double dt;        /* time step */
    double g[3];      /* body-force acceleration */
    double alpha;     /* accommodation: diffuse fraction of the wall (1 in the paper) */
} orc_problem;

enum { FACE_YLO = 0, FACE_YHI = 1, FACE_ZLO = 2, FACE_ZHI = 3 };

static double hermite1(int n, double x)
{
    /* probabilists' Hermite polynomial: the one-dimensional case of defH */
    double hm = 1.0, h = x;
    if (n == 0) return 1.0;
    for (int k = 1; k < n; ++k) {
        double hn = x * h - k * hm;
        hm = h;
        h = hn;
    }
    return h;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= k;
    return f;
}

static void xi_of(const orc_problem *p, int a, double xi[3])
{
    for (int d = 0; d < 3; ++d) xi[d] = p->c * p->e[3 * a + d];
}

/* f^(0)_alpha(rho, u) by the literal tensor contraction over all index tuples */
static double equilibrium_tensor(const orc_problem *p, int a, double rho, const double u[3])
{
    double xi[3];
    xi_of(p, a, xi);
    int D = p->dim;
    double total = 0.0;
    for (int n = 0; n <= p->N; ++n) {
        int idx[16] = {0};
        long count = 1;
        for (int k = 0; k < n; ++k) count *= D;
        double s = 0.0;
        for (long t = 0; t < count; ++t) {
            long r = t;
            int cnt[3] = {0, 0, 0};
            double up = 1.0;
            for (int k = 0; k < n; ++k) {
                idx[k] = (int)(r % D);
                r /= D;
                cnt[idx[k]]++;
                up *= u[idx[k]];
            }
            double h = 1.0;
            for (int d = 0; d < D; ++d) h *= hermite1(cnt[d], xi[d]);
            s += up * h;
        }
        total += s / factorial(n);
    }
    return rho * p->w[a] * total;
}

/* F_alpha of Eq. nm.4; Pi is the 3x3 second moment of f (row-major) or NULL
 * to drop the (Pi - rho I) term (whose second moment vanishes by orthogonality) */
static double force_nm4(const orc_problem *p, int a, double rho, const double u[3],
                        const double *Pi)
{
    double xi[3];
    xi_of(p, a, xi);
    int D = p->dim;
    double gx = 0.0, ux = 0.0, ug = 0.0;
    for (int d = 0; d < D; ++d) {
        gx += p->g[d] * xi[d];
        ux += u[d] * xi[d];
        ug += u[d] * p->g[d];
    }
    double term = gx + (gx * ux - ug);
    if (Pi) {
        double s = 0.0;
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                double a2 = Pi[3 * i + j] - (i == j ? rho : 0.0);
                double h2 = xi[i] * xi[j] - (i == j ? 1.0 : 0.0);
                s += a2 * (gx * h2 - 2.0 * p->g[i] * xi[j]);
            }
        term += s / (2.0 * rho);
    }
    return rho * p->w[a] * term;
}

static long nnodes(const orc_problem *p) { return (long)p->nx * p->ny * p->nz; }

static long node_id(const orc_problem *p, int i, int j, int k)
{
    return ((long)k * p->ny + j) * p->nx + i;
}

static int wrap(int v, int n) { v %= n; return v < 0 ? v + n : v; }

static long face_elems(const orc_problem *p)
{
    long a = (long)p->nx * p->nz, b = (long)p->nx * p->ny;
    return a > b ? a : b;
}

/* Is (j, k) outside the fluid? Sets which directions are out. */
static int outside(const orc_problem *p, int j, int k, int *out_y, int *out_z)
{
    *out_y = (j < 0 || j >= p->ny);
    *out_z = p->walls_z && (k < 0 || k >= p->nz);
    return *out_y || *out_z;
}

/* Fraction of the step at which a particle at coordinate `from`, moving with
 * integer velocity component v != 0, crosses the wall plane ahead of it. */
static double exit_time(double from, int v, int n)
{
    double plane = v > 0 ? (double)n - 0.5 : -0.5;
    return (plane - from) / (double)v;
}

/* Wall face and element of the segment from fluid node (i, j, k) along the
 * outward integer direction (vy, vz) to a point outside the fluid. The face is
 * the first one the segment crosses (ties go to the y face); the element is the
 * fluid node's cell on that face. An emitted slot (x, alpha), whose virtual
 * source x - e_alpha is outside, uses direction -e_alpha; the absorbed
 * population (x, beta) uses +e_beta; so the slot (x, alpha) and the absorbed
 * (x, -alpha) always share face and element. */
static long wall_element(const orc_problem *p, int i, int j, int k, int vy, int vz,
                         int oy, int oz)
{
    int use_z;
    if (oy && oz) {
        double ty = exit_time((double)j, vy, p->ny);
        double tz = exit_time((double)k, vz, p->nz);
        use_z = tz < ty;
    } else {
        use_z = oz;
    }
    long ne = face_elems(p);
    if (use_z) return (long)(vz < 0 ? FACE_ZLO : FACE_ZHI) * ne + (long)j * p->nx + i;
    return (long)(vy < 0 ? FACE_YLO : FACE_YHI) * ne + (long)k * p->nx + i;
}

static double wall_shape(const orc_problem *p, int a)
{
    double xi[3], gx = 0.0;
    xi_of(p, a, xi);
    for (int d = 0; d < p->dim; ++d) gx += p->g[d] * xi[d];
    return p->w[a] * (1.0 - 0.5 * p->dt * gx);
}

/* A(e): post-collision populations leaving through each wall element;
 * D(e): sum of w (1 - dt/2 g.xi) over the unknown slots assigned to e. */
int orc_wall_balance(const orc_problem *p, const double *fpost, double *A, double *Dn)
{
    long ne = face_elems(p);
    memset(A, 0, sizeof(double) * 4 * ne);
    memset(Dn, 0, sizeof(double) * 4 * ne);
    int V = p->V;
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                long n = node_id(p, i, j, k);
                for (int a = 0; a < V; ++a) {
                    int ey = p->e[3 * a + 1], ez = p->e[3 * a + 2];
                    int oy, oz;
                    /* absorbed: destination outside */
                    if (outside(p, j + ey, k + ez, &oy, &oz))
                        A[wall_element(p, i, j, k, ey, ez, oy, oz)] += fpost[n * V + a];
                    /* emitted slot: virtual source outside */
                    if (outside(p, j - ey, k - ez, &oy, &oz))
                        Dn[wall_element(p, i, j, k, -ey, -ez, oy, oz)] += wall_shape(p, a);
                }
            }
    return 0;
}

/* Index of the velocity (e_x, -e_y, e_z) of velocity a. */
static int reflected_y(const orc_problem *p, int a)
{
    for (int b = 0; b < p->V; ++b)
        if (p->e[3 * b] == p->e[3 * a] && p->e[3 * b + 1] == -p->e[3 * a + 1] &&
            p->e[3 * b + 2] == p->e[3 * a + 2])
            return b;
    return -1;
}

/* Streaming pass: fpre(x) = fpost(x - e) inside, wall value otherwise. */
int orc_stream(const orc_problem *p, const double *fpost, double *fpre)
{
    long ne = face_elems(p);
    double *A = (double *)malloc(sizeof(double) * 4 * ne);
    double *Dn = (double *)malloc(sizeof(double) * 4 * ne);
    if (!A || !Dn) { free(A); free(Dn); return -1; }
    orc_wall_balance(p, fpost, A, Dn);
    int V = p->V;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                long n = node_id(p, i, j, k);
                for (int a = 0; a < V; ++a) {
                    int ex = p->e[3 * a], ey = p->e[3 * a + 1], ez = p->e[3 * a + 2];
                    int is = wrap(i - ex, p->nx), js = j - ey, ks = k - ez;
                    int oy, oz;
                    if (!outside(p, js, ks, &oy, &oz)) {
                        if (!p->walls_z) ks = wrap(ks, p->nz);
                        fpre[n * V + a] = fpost[node_id(p, is, js, ks) * V + a];
                    } else {
                        long el = wall_element(p, i, j, k, -ey, -ez, oy, oz);
                        double rho_eff = Dn[el] > 0.0 ? A[el] / Dn[el] : 0.0;
                        double diffuse = rho_eff * wall_shape(p, a);
                        if (p->alpha == 1.0) {
                            fpre[n * V + a] = diffuse;
                        } else {
                            /* image of the source row in the wall plane
                             * y = -1/2 (below) or y = ny - 1/2 (above) */
                            int jm = js < 0 ? -1 - js : 2 * p->ny - 1 - js;
                            int b = reflected_y(p, a);
                            double spec = fpost[node_id(p, is, jm, k) * V + b];
                            fpre[n * V + a] = p->alpha * diffuse + (1.0 - p->alpha) * spec;
                        }
                    }
                }
            }
    free(A);
    free(Dn);
    return 0;
}

/* rho = sum fbar, rho u = sum fbar xi + dt/2 rho g (Eq. nm.10) */
static void node_moments(const orc_problem *p, const double *fb, double *rho, double u[3])
{
    double r = 0.0, j[3] = {0, 0, 0};
    for (int a = 0; a < p->V; ++a) {
        double xi[3];
        xi_of(p, a, xi);
        r += fb[a];
        for (int d = 0; d < 3; ++d) j[d] += fb[a] * xi[d];
    }
    *rho = r;
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * p->dt * r * p->g[d]) / r;
}

int orc_moments(const orc_problem *p, const double *fpre, double *rho, double *u)
{
    long nn = nnodes(p);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < nn; ++n) node_moments(p, fpre + n * p->V, rho + n, u + 3 * n);
    return 0;
}

/* Collision of one node: fbar -> fbar* */
static void collide_node(const orc_problem *p, const double *fb, double *out, double *feq_tmp)
{
    int V = p->V;
    double rho, u[3];
    node_moments(p, fb, &rho, u);
    /* second moment of the physical f from fbar (inverse of Eq. nm.7); the
     * generalised equilibrium's second moment is summed over the DVM with the
     * (Pi - rho I) force term omitted (it is orthogonal to second moments) */
    double S[9] = {0}, Seq[9] = {0};
    for (int a = 0; a < V; ++a) {
        double xi[3];
        xi_of(p, a, xi);
        double feq0 = equilibrium_tensor(p, a, rho, u) + p->tau * force_nm4(p, a, rho, u, NULL);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                S[3 * i + j] += fb[a] * xi[i] * xi[j];
                Seq[3 * i + j] += feq0 * xi[i] * xi[j];
            }
    }
    double h = p->dt / (2.0 * p->tau);
    double Pi[9];
    for (int q = 0; q < 9; ++q) Pi[q] = (S[q] + h * Seq[q]) / (1.0 + h);
    double omega = p->dt / (p->tau + 0.5 * p->dt);
    for (int a = 0; a < V; ++a) {
        double feq = equilibrium_tensor(p, a, rho, u) + p->tau * force_nm4(p, a, rho, u, Pi);
        feq_tmp[a] = feq;
        out[a] = fb[a] - omega * (fb[a] - feq);
    }
}

int orc_collide(const orc_problem *p, const double *fpre, double *fpost)
{
    long nn = nnodes(p);
    int V = p->V;
    int bad = 0;
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * V);
        if (!tmp) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(static)
            for (long n = 0; n < nn; ++n) collide_node(p, fpre + n * V, fpost + n * V, tmp);
        }
        free(tmp);
    }
    return bad ? -1 : 0;
}

/* f = f^(0)(rho(x), u(x)) at every node (u may be NULL for rest) */
int orc_init(const orc_problem *p, const double *rho, const double *u, double *f)
{
    long nn = nnodes(p);
    int V = p->V;
    for (long n = 0; n < nn; ++n) {
        double uu[3] = {0, 0, 0};
        if (u)
            for (int d = 0; d < 3; ++d) uu[d] = u[3 * n + d];
        for (int a = 0; a < V; ++a) f[n * V + a] = equilibrium_tensor(p, a, rho[n], uu);
    }
    return 0;
}

/* n full steps (stream + collide) on the post-collision state f; tmp is a
 * scratch array of the same size */
int orc_run(const orc_problem *p, double *f, double *tmp, long nsteps, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (long s = 0; s < nsteps; ++s) {
        if (orc_stream(p, f, tmp)) return -1;
        if (orc_collide(p, tmp, f)) return -1;
    }
    return 0;
}

/* single-node helpers exposed for the moment-identity tests */
int orc_equilibrium(const orc_problem *p, double rho, const double *u, double *feq)
{
    for (int a = 0; a < p->V; ++a) feq[a] = equilibrium_tensor(p, a, rho, u);
    return 0;
}

int orc_force(const orc_problem *p, double rho, const double *u, const double *Pi, double *F)
{
    for (int a = 0; a < p->V; ++a) F[a] = force_nm4(p, a, rho, u, Pi);
    return 0;
}

int orc_collide_node(const orc_problem *p, const double *fb, double *out)
{
    double *tmp = (double *)malloc(sizeof(double) * p->V);
    if (!tmp) return -1;
    collide_node(p, fb, out, tmp);
    free(tmp);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

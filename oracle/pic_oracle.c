/*
 * pic_oracle.c -- plain, slow, FP64 CPU oracle for one time step of a 1D3V
 * electrostatic Particle-in-Cell Monte Carlo (PIC-MC) code.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code with the
 * GPU library: no header, helper, table or constant generator.
 *
 * What it follows (Williams et al., "Accelerating Particle-in-Cell Monte
 * Carlo Simulations with MPI, OpenMP/OpenACC and Asynchronous Multi-GPU
 * Programming", arXiv 2404.10270):
 *   - Sec. 2, the five-phase explicit PIC cycle: charge deposition with
 *     interpolation functions, (smoother), Poisson solve with a tridiagonal
 *     matrix and E = -grad(phi), Monte Carlo collisions and plasma-wall
 *     interaction, and the mover dv/dt = (q/m) E, dx/dt = v;
 *   - Sec. 6, the moveb listing: linear gather a[j] + x (a[j+1] - a[j]) with
 *     the in-cell coordinate x, velocity kick, position advance x += nstep*vx;
 *   - Sec. 2, "natural sorting" (particles grouped by cell): the oracle never
 *     needs it, every result here is independent of particle order;
 *   - Sec. 3.4 (Table 1 and the text after it), the test case: electrons,
 *     D+ ions and kinetic D atoms, no field solver, electron-atom elastic,
 *     excitation and ionisation, the gas depleting by dn/dt = -n n_e R.
 * Where the paper is silent (magnetised Boris rotation, the null-collision
 * Monte Carlo, Philox draws keyed by particle id and step, fixed-point
 * deposition, wall-node closure, the pair source and ids of created
 * particles) each function states the reading it implements.
 *
 * Units: positions in cells, velocities in cells per step; the physical
 * inputs (SI or plasma units) are converted here, independently of the GPU
 * library.  Everything is FP64; build with -ffp-contract=off so that no
 * multiply-add is fused unless fma() is written out.
 *
 * Threads (OpenMP, orc_set_threads; one by default): only loops whose
 * iterations are independent run in parallel -- the push of each particle,
 * the periodic wrap, the collision-candidate draw of each particle, and the
 * deposit into per-thread integer arrays that are then added (integer sums
 * do not depend on order).  Collisions, walls, source, field and the
 * floating-point sums of the diagnostics stay serial in particle order, so
 * every result is bit-identical for any thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXSP 4
#define ORC_FRAC_BITS 32            /* fixed-point fraction bits of the deposit */
#define ORC_KIND_ELECTRON 0
#define ORC_KIND_ION 1
#define ORC_KIND_NEUTRAL 2          /* kinetic neutral (q = 0): moved ballistically, ionised */
#define ORC_XS_IZ_RATE 1u           /* ionisation with a constant rate coefficient sig_iz v_cap */
#define ORC_BC_PERIODIC 0
#define ORC_BC_ABSORB 1

#define ORC_ST_CAPACITY 1u          /* an append did not fit: the particle was dropped */
#define ORC_ST_CFL 2u               /* |vx| >= 1 cell per step */
#define ORC_ST_NN_CAP 4u            /* a local neutral density exceeded the bound n_n */

typedef struct {
    int32_t nc, bc, nsp, mcc_on, source_on, inst;
    uint64_t seed;
    double dx, dt, eps0, B0, theta;
    double q[ORC_MAXSP], m[ORC_MAXSP], w[ORC_MAXSP];
    int32_t kind[ORC_MAXSP];
    int32_t nstep[ORC_MAXSP];       /* push every nstep steps (subcycling); 0 or 1 = every step */
    double v_cap[ORC_MAXSP];        /* m/s */
    double T_src[ORC_MAXSP];        /* J */
    double n_n, T_n, sig_el, sig_iz, E_iz, sig_cx;
    int32_t smooth_passes, _pad;    /* density smoother (0 = off) */
    double sig_ex, E_ex;            /* electron-impact excitation: cross section, threshold */
    int32_t field_off;              /* no field solve: E = 0 (the paper's Table 1 case) */
    uint32_t xs_flags;              /* ORC_XS_* */
} orc_config;

typedef struct {
    int64_t n, cap;
    double *x, *vx, *vy, *vz;
    uint64_t *id;
} orc_particles;

typedef struct {
    int64_t step;
    uint64_t next_id;
    uint32_t status, _pad;
    int64_t absorbed[ORC_MAXSP][2];        /* this step, [left, right] wall */
    int64_t absorbed_total[ORC_MAXSP][2];
    int64_t created_total[ORC_MAXSP];
    int64_t n_candidates, n_elastic, n_ionize, n_cx, n_over_cap, n_source;  /* totals */
    int64_t particle_steps;
    int64_t n_excite, n_consumed, n_iz_untargeted;  /* totals (kinetic neutrals) */
} orc_counters;

typedef struct {
    orc_config cfg;
    orc_particles sp[ORC_MAXSP];
    orc_counters cnt;
    uint64_t *S[ORC_MAXSP];     /* nc+1 fixed-point deposit per species */
    double *rho, *phi, *E;      /* nc+1 */
    double *acc[ORC_MAXSP];     /* nc+1, cells / step^2 */
    double *nn;                 /* nc+1, density of the kinetic neutral species [m^-3] */
} orc_sim;

typedef struct {
    int64_t n[ORC_MAXSP];
    double ke[ORC_MAXSP];          /* sum 1/2 m w |V|^2  [J / m^2] */
    double mom[ORC_MAXSP][3];      /* sum m w V          [kg / (m s)] */
    double field_energy;           /* 1/2 eps0 sum E_j^2 V_j [J / m^2] */
} orc_diag;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Each round multiplies counter words 0 and 2 by */
/* fixed odd constants, takes the high and low halves of the 64-bit products */
/* and mixes them with words 1, 3 and the key; the key is bumped by the two  */
/* Weyl constants between rounds.                                             */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform on (0,1): (u + 1/2) 2^-32, exact in FP64 */
static double u01(uint32_t u) { return ((double)u + 0.5) * 0x1p-32; }

/* the first species of a kind (electron, ion, kinetic neutral), or -1 */
static int find_kind(const orc_config *c, int kind)
{
    for (int k = 0; k < c->nsp; ++k) if (c->kind[k] == kind) return k;
    return -1;
}

static void draw_block(const orc_config *c, uint64_t id, int64_t step, uint32_t block,
                       uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), (uint32_t)step, block};
    uint32_t key[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32) ^ (uint32_t)c->inst};
    orc_philox4x32_10(ctr, key, out);
}

/* source pair k draws: counter word 1 = 0xFFFFFFFF, which no particle id
 * (all ids are below 2^63) ever has */
static void draw_block_source(const orc_config *c, uint64_t k, int64_t step, uint32_t block,
                              uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)k, 0xFFFFFFFFu, (uint32_t)step, block};
    uint32_t key[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32) ^ (uint32_t)c->inst};
    orc_philox4x32_10(ctr, key, out);
}

/* Box-Muller: two uniforms -> two standard normals */
static void box_muller(uint32_t a, uint32_t b, double *n0, double *n1)
{
    double r = sqrt(-2.0 * log(u01(a)));
    double t = 2.0 * M_PI * u01(b);
    *n0 = r * cos(t);
    *n1 = r * sin(t);
}

/* isotropic unit vector from two uniforms: cos(chi) = 1 - 2 U, phi = 2 pi U' */
static void iso_dir(uint32_t a, uint32_t b, double d[3])
{
    double cc = 1.0 - 2.0 * u01(a);
    double ss = sqrt(fmax(0.0, 1.0 - cc * cc));
    double ph = 2.0 * M_PI * u01(b);
    d[0] = cc;
    d[1] = ss * cos(ph);
    d[2] = ss * sin(ph);
}

/* ------------------------------------------------------------------------ */
/* Phase 1: charge deposition (Sec. 2, "plasma density calculation").        */
/* Linear (cloud-in-cell) weights, the same interpolation the moveb gather   */
/* uses.  Fixed point with F = 32 fraction bits: the right node receives     */
/* W1 = rint(f 2^32) and the left node 2^32 - W1, so every particle adds     */
/* exactly 2^32 and the sum is independent of order.                          */
/* ------------------------------------------------------------------------ */
/* add one particle at x (cells) to the fixed-point deposit S */
static void deposit_add(double x, uint64_t *S)
{
    double jd = floor(x);
    double f = x - jd;
    int64_t j = (int64_t)jd;
    uint64_t w1 = (uint64_t)rint(ldexp(f, ORC_FRAC_BITS));
    S[j] += ((uint64_t)1 << ORC_FRAC_BITS) - w1;
    S[j + 1] += w1;
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_deposit_species(int64_t n, const double *x, int32_t nc, uint64_t *S)
{
    const size_t G = (size_t)nc + 1;
    memset(S, 0, sizeof(uint64_t) * G);
    int nt = orc_get_threads();
    /* each thread deposits its share into an array of its own; the integer
     * arrays are then added, which gives the same S in any order */
    uint64_t *T = nt > 1 ? (uint64_t *)calloc((size_t)nt * G, sizeof(uint64_t)) : NULL;
    if (!T) {
        for (int64_t p = 0; p < n; ++p) deposit_add(x[p], S);
        return;
    }
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        uint64_t *Tt = T + (size_t)omp_get_thread_num() * G;
#else
        uint64_t *Tt = T;
#endif
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) deposit_add(x[p], Tt);
    }
    for (int t = 0; t < nt; ++t)
        for (size_t j = 0; j < G; ++j) S[j] += T[(size_t)t * G + j];
    free(T);
}

/* the same linear weights in plain FP64 (used to bound the fixed-point error) */
void orc_deposit_cic64(int64_t n, const double *x, int32_t nc, double *out)
{
    memset(out, 0, sizeof(double) * (size_t)(nc + 1));
    for (int64_t p = 0; p < n; ++p) {
        double jd = floor(x[p]);
        double f = x[p] - jd;
        int64_t j = (int64_t)jd;
        out[j] += 1.0 - f;
        out[j + 1] += f;
    }
}

void orc_deposit(orc_sim *s)
{
    for (int k = 0; k < s->cfg.nsp; ++k)
        orc_deposit_species(s->sp[k].n, s->sp[k].x, s->cfg.nc, s->S[k]);
}

/* ------------------------------------------------------------------------ */
/* Phase 3: field solve (Sec. 2).  Textbook Thomas algorithm for            */
/* a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, i = 0..n-1 (a_0 and c_{n-1}     */
/* unused).                                                                   */
/* ------------------------------------------------------------------------ */
int orc_thomas(int64_t n, const double *a, const double *b, const double *c, const double *d,
               double *x)
{
    if (n <= 0) return 0;
    double *cp = (double *)malloc(sizeof(double) * (size_t)n);
    double *dp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!cp || !dp) { free(cp); free(dp); return -1; }
    cp[0] = c[0] / b[0];
    dp[0] = d[0] / b[0];
    for (int64_t i = 1; i < n; ++i) {
        double den = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / den;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    free(cp);
    free(dp);
    return 0;
}

/*
 * rho from the fixed-point deposits, Poisson  phi_{j-1} - 2 phi_j + phi_{j+1}
 * = -rho_j dx^2 / eps0 by Thomas, E = -grad(phi), and the per-species grid
 * acceleration acc_s = (q_s/m_s) E dt^2 / dx (cells per step^2).
 *
 * Absorbing walls (grounded, phi_0 = phi_nc = 0): the wall nodes own half a
 * cell (V = dx/2), interior E is the central difference, and the wall E
 * closes Gauss's law over the half cell: E_0 = -(phi_1 - phi_0)/dx -
 * rho_0 dx/(2 eps0), E_nc = -(phi_nc - phi_{nc-1})/dx + rho_nc dx/(2 eps0).
 *
 * Periodic: node nc is node 0 (its deposit is folded onto node 0), an
 * immobile uniform background rho_bg = -sum_s q_s w_s N_s / (nc dx) makes
 * the system neutral, and the gauge phi_0 = 0 leaves the same tridiagonal
 * system on nodes 1..nc-1.
 */
/* Thomas algorithm for the Dirichlet Poisson matrix tridiag(1, -2, 1) of n
 * unknowns (Sec. 2, field solver).  Its pivots are known in closed form: the
 * elimination leaves den_u = -(u+1)/u on the diagonal and c'_u = -u/(u+1)
 * above it (u = 1..n).  They are evaluated from that form rather than by the
 * recurrence den_u = -2 - c'_{u-1}: the recurrence sits on a neutrally
 * stable fixed point, so its rounding errors do not decay and at 10^6 cells
 * they move phi by ~5e-7 of its maximum; the closed form is exact to one
 * rounding per pivot. */
int orc_poisson_dirichlet(int64_t n, const double *d, double *x)
{
    if (n <= 0) return 0;
    double *dp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!dp) return -1;
    double prev = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double u = (double)(i + 1);
        const double den = -(u + 1.0) / u;
        prev = (d[i] - prev) / den;
        dp[i] = prev;
    }
    x[n - 1] = dp[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) {
        const double u = (double)(i + 1);
        const double cp = -u / (u + 1.0);
        x[i] = dp[i] - cp * x[i + 1];
    }
    free(dp);
    return 0;
}

/* Density smoother (Sec. 2, phase 2).  The paper names the phase but gives
 * no stencil; one pass here is the binomial (1, 2, 1)/4 filter applied to the
 * node charges Q_j = rho_j V_j: every node keeps half of its charge and
 * passes a quarter to each neighbour.  At an absorbing wall the quarter that
 * would leave the domain stays on the wall node, so the total charge is
 * unchanged; a periodic grid wraps (node nc is node 0).  rho is read and
 * written in place, V holds the node volumes. */
void orc_smooth(int32_t nc, int bc, int passes, const double *V, double *rho)
{
    const int32_t n = (bc == ORC_BC_PERIODIC) ? nc : nc + 1;  /* distinct nodes */
    double *Q = (double *)malloc(sizeof(double) * (size_t)n);
    double *R = (double *)malloc(sizeof(double) * (size_t)n);
    if (!Q || !R) { free(Q); free(R); return; }
    for (int32_t j = 0; j < n; ++j) Q[j] = rho[j] * V[j];
    for (int p = 0; p < passes; ++p) {
        for (int32_t j = 0; j < n; ++j) {
            double left, right;
            if (bc == ORC_BC_PERIODIC) {
                left = Q[(j + n - 1) % n];
                right = Q[(j + 1) % n];
            } else {
                left = j > 0 ? Q[j - 1] : Q[j];
                right = j < n - 1 ? Q[j + 1] : Q[j];
            }
            R[j] = (left + 2.0 * Q[j] + right) * 0.25;
        }
        double *t = Q; Q = R; R = t;
    }
    for (int32_t j = 0; j < n; ++j) rho[j] = Q[j] / V[j];
    if (bc == ORC_BC_PERIODIC) rho[nc] = rho[0];
    free(Q);
    free(R);
}

int orc_field(orc_sim *s)
{
    const orc_config *c = &s->cfg;
    const int32_t nc = c->nc;
    const double dx = c->dx;
    double *rho = s->rho, *phi = s->phi, *E = s->E;
    const double two_m32 = 0x1p-32;

    double rho_bg = 0.0;
    if (c->bc == ORC_BC_PERIODIC) {
        double qn = 0.0;
        for (int k = 0; k < c->nsp; ++k) qn += (c->q[k] * c->w[k]) * (double)s->sp[k].n;
        rho_bg = -qn / ((double)nc * dx);
    }
    for (int32_t j = 0; j <= nc; ++j) {
        double acc = 0.0;
        for (int k = 0; k < c->nsp; ++k) {
            uint64_t Sj = s->S[k][j];
            if (c->bc == ORC_BC_PERIODIC) {
                if (j == 0) Sj += s->S[k][nc];
                if (j == nc) Sj = s->S[k][0] + s->S[k][nc];
            }
            acc += (c->q[k] * c->w[k]) * ((double)Sj * two_m32);
        }
        double V = dx;
        if (c->bc == ORC_BC_ABSORB && (j == 0 || j == nc)) V = 0.5 * dx;
        rho[j] = acc / V + rho_bg;
    }
    /* density of the kinetic neutral species at the nodes, from its deposit
     * with the same node volumes: real neutrals per macro-particle per unit
     * area times the deposited particle count, over the node volume */
    if (s->nn) {
        const int kn = find_kind(c, ORC_KIND_NEUTRAL);
        for (int32_t j = 0; j <= nc; ++j) {
            double n = 0.0;
            if (kn >= 0) {
                uint64_t Sj = s->S[kn][j];
                if (c->bc == ORC_BC_PERIODIC) {
                    if (j == 0) Sj += s->S[kn][nc];
                    if (j == nc) Sj = s->S[kn][0] + s->S[kn][nc];
                }
                double V = dx;
                if (c->bc == ORC_BC_ABSORB && (j == 0 || j == nc)) V = 0.5 * dx;
                n = (c->w[kn] * ((double)Sj * two_m32)) / V;
            }
            s->nn[j] = n;
        }
    }
    /* the paper's Table 1 case runs without the field solver: E = 0 */
    if (c->field_off) {
        for (int32_t j = 0; j <= nc; ++j) phi[j] = E[j] = 0.0;
        for (int k = 0; k < c->nsp; ++k)
            for (int32_t j = 0; j <= nc; ++j) s->acc[k][j] = 0.0;
        return 0;
    }
    if (c->smooth_passes > 0) {
        double *Vn = (double *)malloc(sizeof(double) * (size_t)(nc + 1));
        if (!Vn) return -1;
        for (int32_t j = 0; j <= nc; ++j)
            Vn[j] = (c->bc == ORC_BC_ABSORB && (j == 0 || j == nc)) ? 0.5 * dx : dx;
        orc_smooth(nc, c->bc, c->smooth_passes, Vn, rho);
        free(Vn);
    }

    /* unknowns phi_1 .. phi_{nc-1} */
    const int64_t n = nc - 1;
    const double K = dx * dx / c->eps0;
    phi[0] = 0.0;
    phi[nc] = 0.0;
    if (n > 0) {
        double *d = (double *)malloc(sizeof(double) * (size_t)n);
        if (!d) return -1;
        for (int64_t i = 0; i < n; ++i) d[i] = -(rho[i + 1] * K);
        int rc = orc_poisson_dirichlet(n, d, phi + 1);
        free(d);
        if (rc) return rc;
    }

    for (int32_t j = 1; j < nc; ++j) E[j] = (phi[j - 1] - phi[j + 1]) / (2.0 * dx);
    if (c->bc == ORC_BC_ABSORB) {
        E[0] = -(phi[1] - phi[0]) / dx - rho[0] * dx / (2.0 * c->eps0);
        E[nc] = -(phi[nc] - phi[nc - 1]) / dx + rho[nc] * dx / (2.0 * c->eps0);
    } else {
        E[0] = (phi[nc - 1] - phi[1]) / (2.0 * dx);
        E[nc] = E[0];
    }
    for (int k = 0; k < c->nsp; ++k) {
        const double C = (c->q[k] / c->m[k]) * (c->dt * c->dt / dx);
        for (int32_t j = 0; j <= nc; ++j) s->acc[k][j] = C * E[j];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Phase 5: mover (Sec. 2 and the moveb listing of Sec. 6).                   */
/* Gather a = a[j] + f (a[j+1] - a[j]) with in-cell f (written as one fma),   */
/* then a Boris step for the magnetised 1D3V case: half electric kick,        */
/* rotation about B with t = (q/m) B dt/2 and s = 2t/(1+|t|^2), second half   */
/* kick; then the advance x += vx (nstep = 1).  B = B0 (cos th, sin th, 0),   */
/* th measured from the wall normal x.                                        */
/* ------------------------------------------------------------------------ */
/* Subcycling (the per-species step multiplier nstep of the moveb listing,
 * Sec. 6): species k is pushed only on steps s with s mod nstep = 0, over a
 * time nstep dt -- the kick, the rotation angle and the advance
 * x += nstep vx all take nstep dt; its particles keep their positions (and
 * their deposit) on the steps in between, and its collision test runs on
 * the push steps with the probability of nstep dt. */
static int sub_of(const orc_config *c, int k) { return c->nstep[k] > 1 ? c->nstep[k] : 1; }

static int pushed_at(const orc_config *c, int k, int64_t step) { return step % sub_of(c, k) == 0; }

static void species_rotation(const orc_config *c, int k, double t[2], double sv[2])
{
    const double tm = (c->q[k] / c->m[k]) * c->B0 * (0.5 * (c->dt * (double)sub_of(c, k)));
    t[0] = tm * cos(c->theta);
    t[1] = tm * sin(c->theta);
    const double den = 1.0 + (t[0] * t[0] + t[1] * t[1]);
    sv[0] = 2.0 * t[0] / den;
    sv[1] = 2.0 * t[1] / den;
}

void orc_push_species(const orc_config *c, int k, const double *acc, int64_t n, double *x,
                      double *vx, double *vy, double *vz)
{
    double t[2], sv[2];
    species_rotation(c, k, t, sv);
    const double tx = t[0], ty = t[1], sx = sv[0], sy = sv[1];
    const double ms = (double)sub_of(c, k);
    const double hk = 0.5 * ms;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double jd = floor(x[p]);
        double f = x[p] - jd;
        int64_t j = (int64_t)jd;
        double a = fma(f, acc[j + 1] - acc[j], acc[j]);
        double h = hk * a;
        double mx = vx[p] + h, my = vy[p], mz = vz[p];
        /* v' = v- + v- x t,  t = (tx, ty, 0) */
        double px = mx - mz * ty;
        double py = my + mz * tx;
        double pz = mz + (mx * ty - my * tx);
        /* v+ = v- + v' x s,  s = (sx, sy, 0) */
        double qx = mx - pz * sy;
        double qy = my + pz * sx;
        double qz = mz + (px * sy - py * sx);
        vx[p] = qx + h;
        vy[p] = qy;
        vz[p] = qz;
        x[p] = x[p] + ms * vx[p];
    }
}

void orc_push(orc_sim *s)
{
    for (int k = 0; k < s->cfg.nsp; ++k) {
        if (!pushed_at(&s->cfg, k, s->cnt.step)) continue;
        orc_particles *P = &s->sp[k];
        orc_push_species(&s->cfg, k, s->acc[k], P->n, P->x, P->vx, P->vy, P->vz);
        const double ms = (double)sub_of(&s->cfg, k);
        int cfl = 0;
#pragma omp parallel for schedule(static) reduction(| : cfl)
        for (int64_t p = 0; p < P->n; ++p)
            if (fabs(ms * P->vx[p]) >= 1.0) cfl = 1;
        if (cfl) s->cnt.status |= ORC_ST_CFL;
        s->cnt.particle_steps += P->n;
    }
}

/* ------------------------------------------------------------------------ */
/* Plasma-wall interaction (Sec. 2, phase 4): grounded absorbing walls at     */
/* x = 0 and x = nc (a particle at x < 0 or x >= nc is removed and counted    */
/* per wall), or periodic re-entry with the same velocity (Table 1).          */
/* ------------------------------------------------------------------------ */
void orc_walls(orc_sim *s)
{
    const orc_config *c = &s->cfg;
    const double L = (double)c->nc;
    for (int k = 0; k < c->nsp; ++k) {
        orc_particles *P = &s->sp[k];
        s->cnt.absorbed[k][0] = s->cnt.absorbed[k][1] = 0;
        if (c->bc == ORC_BC_PERIODIC) {
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < P->n; ++p) {
                double x = P->x[p];
                if (x < 0.0) x += L;
                else if (x >= L) x -= L;
                if (x >= L) x -= L;
                P->x[p] = x;
            }
            continue;
        }
        int64_t keep = 0;
        for (int64_t p = 0; p < P->n; ++p) {
            double x = P->x[p];
            if (x < 0.0) { s->cnt.absorbed[k][0]++; continue; }
            if (x >= L) { s->cnt.absorbed[k][1]++; continue; }
            P->x[keep] = x;
            P->vx[keep] = P->vx[p];
            P->vy[keep] = P->vy[p];
            P->vz[keep] = P->vz[p];
            P->id[keep] = P->id[p];
            keep++;
        }
        P->n = keep;
        s->cnt.absorbed_total[k][0] += s->cnt.absorbed[k][0];
        s->cnt.absorbed_total[k][1] += s->cnt.absorbed[k][1];
    }
}

/* ------------------------------------------------------------------------ */
/* Collisions (Sec. 2, phase 4: Monte Carlo collisions and ionisation).       */
/* Null-collision method (Vahedi & Surendra, CPC 87, 1995) against a uniform  */
/* cold-rate neutral gas of density n_n: per species the collision frequency  */
/* is bounded by nu_max = n_n sum_k sigma_k v_cap, a particle is a candidate  */
/* with probability P = 1 - exp(-nu_max dt), tested as u0 < floor(P 2^32),    */
/* and a candidate undergoes process k iff r = U(u1) nu_max falls below the   */
/* cumulative n_n sigma |v| (ionisation only above its threshold energy).     */
/* All rates in cells and steps: nu dt = n_n sigma dx |v_hat|.                */
/* Draw block b of a particle is Philox(ctr = (id_lo, id_hi, step, b),        */
/* key = (seed_lo, seed_hi ^ instance)).                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t parent;
    double x;              /* parent position (cells) */
    int64_t cell;          /* parent cell */
    double ve[3], vi[3];   /* the new electron; the new ion's Maxwellian draw */
    int64_t target;        /* kinetic neutral consumed by the event, or -1 */
} orc_iz_event;

static int cmp_event(const void *a, const void *b)
{
    uint64_t pa = ((const orc_iz_event *)a)->parent, pb = ((const orc_iz_event *)b)->parent;
    return (pa > pb) - (pa < pb);
}

static int append(orc_sim *s, int k, double x, const double v[3], uint64_t id)
{
    orc_particles *P = &s->sp[k];
    if (P->n >= P->cap) { s->cnt.status |= ORC_ST_CAPACITY; return 0; }
    P->x[P->n] = x;
    P->vx[P->n] = v[0];
    P->vy[P->n] = v[1];
    P->vz[P->n] = v[2];
    P->id[P->n] = id;
    P->n++;
    s->cnt.created_total[k]++;
    return 1;
}

/* threshold T = floor(P 2^32) of the candidate test, 0 <= T <= 2^32 */
/* threshold T = floor(P 2^32) of the candidate test, 0 <= T <= 2^32.  The
 * electron bound sums elastic, excitation and ionisation; with a constant
 * ionisation rate coefficient sig_iz v_cap its term is bounded the same way.
 * A kinetic neutral takes no test. */
uint64_t orc_candidate_threshold(const orc_config *c, int k)
{
    const double dx = c->dx, dt = c->dt;
    double sig = 0.0;
    if (c->kind[k] == ORC_KIND_ELECTRON) sig = (c->sig_el + c->sig_ex) + c->sig_iz;
    else if (c->kind[k] == ORC_KIND_ION) sig = c->sig_cx;
    double vcap_hat = c->v_cap[k] * (dt / dx);
    double nu_max = c->n_n * sig * dx * vcap_hat;       /* per step */
    double P = -expm1(-(nu_max * (double)sub_of(c, k)));  /* per push */
    double T = floor(ldexp(P, 32));
    if (T > 4294967296.0) T = 4294967296.0;
    return (uint64_t)T;
}

/* density of the kinetic neutrals at x (cells): the node densities of the
 * last field pass, gathered with the mover's linear weights */
static double neutral_density_at(const orc_sim *s, double x)
{
    const double jd = floor(x);
    const double f = x - jd;
    const int64_t j = (int64_t)jd;
    return fma(f, s->nn[j + 1] - s->nn[j], s->nn[j]);
}

/* ------------------------------------------------------------------------ */
/* Kinetic neutrals (the paper's Table 1 case, Sec. 3.4: electron-impact      */
/* ionisation depletes the gas).  An ionisation event takes its neutral from  */
/* the parent electron's cell: the events of one cell, in parent-id order,    */
/* consume that cell's live neutrals (positions after this step's push) in    */
/* the order of a key drawn for each neutral from block 3 of its own counter, */
/* (key, id) ascending.  The new ion is the consumed atom: it takes the       */
/* neutral's position and velocity.  Events beyond the neutrals of their cell */
/* consume nothing and keep the Maxwellian ion at the parent.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t cell;
    uint64_t key, id;
    int64_t idx;
} orc_nkey;

static int cmp_nkey(const void *a, const void *b)
{
    const orc_nkey *p = (const orc_nkey *)a, *q = (const orc_nkey *)b;
    if (p->cell != q->cell) return (p->cell > q->cell) - (p->cell < q->cell);
    if (p->key != q->key) return (p->key > q->key) - (p->key < q->key);
    return (p->id > q->id) - (p->id < q->id);
}

uint64_t orc_neutral_key(const orc_config *c, uint64_t id, int64_t step)
{
    uint32_t u[4];
    draw_block(c, id, step, 3, u);
    return ((uint64_t)u[0] << 32) | (uint64_t)u[1];
}

static int consume_neutrals(orc_sim *s, int kn, orc_iz_event *ev, int64_t n_ev)
{
    const orc_config *c = &s->cfg;
    orc_particles *N = &s->sp[kn];
    const int32_t nc = c->nc;
    const int64_t step = s->cnt.step;
    int64_t *want = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    int64_t *gbeg = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    int64_t *used = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    orc_nkey *list = (orc_nkey *)malloc(sizeof(orc_nkey) * (size_t)(N->n > 0 ? N->n : 1));
    unsigned char *dead = (unsigned char *)calloc((size_t)(N->n > 0 ? N->n : 1), 1);
    if (!want || !gbeg || !used || !list || !dead) {
        free(want); free(gbeg); free(used); free(list); free(dead);
        return -1;
    }
    for (int64_t r = 0; r < n_ev; ++r) want[ev[r].cell]++;
    /* the live neutrals of the cells with events, grouped by cell, keyed */
    int64_t m = 0;
    for (int64_t i = 0; i < N->n; ++i) {
        const int64_t j = (int64_t)floor(N->x[i]);
        if (want[j] == 0) continue;
        list[m].cell = j;
        list[m].key = orc_neutral_key(c, N->id[i], step);
        list[m].id = N->id[i];
        list[m].idx = i;
        m++;
    }
    if (m > 1) qsort(list, (size_t)m, sizeof(orc_nkey), cmp_nkey);
    for (int32_t j = 0; j < nc; ++j) gbeg[j] = -1;
    for (int64_t q = m - 1; q >= 0; --q) gbeg[list[q].cell] = q;
    /* events in parent-id order take the neutrals of their cell in key order */
    for (int64_t r = 0; r < n_ev; ++r) {
        const int64_t j = ev[r].cell;
        const int64_t q = used[j]++;
        ev[r].target = -1;
        if (gbeg[j] >= 0 && gbeg[j] + q < m && list[gbeg[j] + q].cell == j) {
            const int64_t i = list[gbeg[j] + q].idx;
            ev[r].target = i;
            dead[i] = 1;
            ev[r].vi[0] = N->vx[i];
            ev[r].vi[1] = N->vy[i];
            ev[r].vi[2] = N->vz[i];
            s->cnt.n_consumed++;
        } else {
            s->cnt.n_iz_untargeted++;
        }
    }
    /* positions of the consumed atoms for their ions, then remove them */
    for (int64_t r = 0; r < n_ev; ++r)
        if (ev[r].target >= 0) ev[r].x = N->x[ev[r].target];
    int64_t keep = 0;
    for (int64_t i = 0; i < N->n; ++i) {
        if (dead[i]) continue;
        N->x[keep] = N->x[i];
        N->vx[keep] = N->vx[i];
        N->vy[keep] = N->vy[i];
        N->vz[keep] = N->vz[i];
        N->id[keep] = N->id[i];
        keep++;
    }
    N->n = keep;
    free(want); free(gbeg); free(used); free(list); free(dead);
    return 0;
}

int orc_mcc(orc_sim *s)
{
    const orc_config *c = &s->cfg;
    if (!c->mcc_on) return 0;
    const double dx = c->dx, dt = c->dt;
    const int ke = find_kind(c, ORC_KIND_ELECTRON), ki = find_kind(c, ORC_KIND_ION);
    const int kn = find_kind(c, ORC_KIND_NEUTRAL);
    if (ke < 0 || ki < 0) return -1;
    if (kn >= 0 && (c->sig_cx != 0.0 || !s->nn)) return -1;  /* no ion-neutral processes here */
    const double M = kn >= 0 ? c->m[kn] : c->m[ki];  /* neutral mass (elastic target) */
    const int rate_iz = (c->xs_flags & ORC_XS_IZ_RATE) != 0;
    const int64_t step = s->cnt.step;

    orc_iz_event *ev = NULL;
    int64_t n_ev = 0;
    if (s->sp[ke].n > 0) {
        ev = (orc_iz_event *)malloc(sizeof(orc_iz_event) * (size_t)s->sp[ke].n);
        if (!ev) return -1;
    }

    for (int k = 0; k < c->nsp; ++k) {
        if (!pushed_at(c, k, step)) continue;  /* tested on its push steps only */
        if (c->kind[k] == ORC_KIND_NEUTRAL) continue;
        orc_particles *P = &s->sp[k];
        const int is_e = (c->kind[k] == ORC_KIND_ELECTRON);
        const uint64_t T = orc_candidate_threshold(c, k);
        const double vcap_hat = c->v_cap[k] * (dt / dx);
        /* the bound nu_max from n_n (the uniform gas, or the bound of the
         * local density of kinetic neutrals) */
        const double sig_tot = is_e ? (c->sig_el + c->sig_ex) + c->sig_iz : c->sig_cx;
        const double nu_max = ((c->n_n * sig_tot) * dx) * vcap_hat;
        const double vcap2 = vcap_hat * vcap_hat;
        /* threshold speeds^2 in (cells/step)^2: 2 E / m_e (dt/dx)^2 */
        const double v2_iz = (2.0 * c->E_iz / c->m[k]) * ((dt / dx) * (dt / dx));
        const double v2_ex = (2.0 * c->E_ex / c->m[k]) * ((dt / dx) * (dt / dx));
        const double eps_iz = 0.5 * v2_iz;
        /* neutral thermal speed (cells/step) for Maxwellian products */
        const double sig_n = sqrt(c->T_n / M) * (dt / dx);
        const double am = c->m[k] / (c->m[k] + M), bm = M / (c->m[k] + M);
        /* the candidate test of each particle depends on its own draw only:
         * it runs in parallel; the candidates then collide in particle order */
        uint8_t *cand = P->n > 0 ? (uint8_t *)malloc((size_t)P->n) : NULL;
        if (P->n > 0 && !cand) { free(ev); return -1; }
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < P->n; ++p) {
            uint32_t u[4];
            draw_block(c, P->id[p], step, 0, u);
            cand[p] = (uint64_t)u[0] < T;
        }
        for (int64_t p = 0; p < P->n; ++p) {
            if (!cand[p]) continue;
            uint32_t u[4];
            draw_block(c, P->id[p], step, 0, u);
            s->cnt.n_candidates++;
            const double vx = P->vx[p], vy = P->vy[p], vz = P->vz[p];
            const double v2 = (vx * vx + vy * vy) + vz * vz;
            if (v2 > vcap2) s->cnt.n_over_cap++;
            /* the neutral density the candidate sees */
            double nl = c->n_n;
            if (kn >= 0) {
                nl = neutral_density_at(s, P->x[p]);
                if (nl > c->n_n) s->cnt.status |= ORC_ST_NN_CAP;
            }
            /* cumulative (density x cross section x dx) of the processes */
            double c0, c1, c2;
            if (is_e) {
                c0 = (nl * c->sig_el) * dx;
                c1 = (nl * (c->sig_el + c->sig_ex)) * dx;
                c2 = (nl * ((c->sig_el + c->sig_ex) + c->sig_iz)) * dx;
            } else {
                c0 = (nl * c->sig_cx) * dx;
                c1 = c0;
                c2 = c0;
            }
            const double C0 = c0 * c0, C1 = c1 * c1, C2 = c2 * c2;
            const double r = u01(u[1]) * nu_max;
            const double r2 = r * r;
            if (is_e) {
                int iz = 0;
                if (r2 < C0 * v2) {
                    /* elastic, cold neutral target, isotropic in the centre of mass */
                    double d[3];
                    iso_dir(u[2], u[3], d);
                    const double g = sqrt(v2);
                    P->vx[p] = am * vx + bm * g * d[0];
                    P->vy[p] = am * vy + bm * g * d[1];
                    P->vz[p] = am * vz + bm * g * d[2];
                    s->cnt.n_elastic++;
                } else if (r2 < C1 * v2) {
                    /* excitation above its threshold: the electron loses E_ex
                     * and leaves isotropically (the atom is not followed) */
                    if (v2 >= v2_ex) {
                        double d[3];
                        iso_dir(u[2], u[3], d);
                        const double g = sqrt(v2 - v2_ex);
                        P->vx[p] = g * d[0];
                        P->vy[p] = g * d[1];
                        P->vz[p] = g * d[2];
                        s->cnt.n_excite++;
                    }
                } else if (v2 >= v2_iz) {
                    if (rate_iz) {
                        /* slot width nl sig_iz dx v_cap: r < c1 |v| + that */
                        const double rr = r - ((nl * c->sig_iz) * dx) * vcap_hat;
                        iz = rr < 0.0 || rr * rr < C1 * v2;
                    } else {
                        iz = r2 < C2 * v2;
                    }
                }
                if (iz) {
                    /* ionisation: the energy above threshold is split U : 1-U
                     * between the two electrons, both isotropic; the new ion
                     * takes a neutral's Maxwellian velocity (or, with kinetic
                     * neutrals, the consumed atom's) */
                    uint32_t u1[4], u2[4];
                    draw_block(c, P->id[p], step, 1, u1);
                    draw_block(c, P->id[p], step, 2, u2);
                    const double e_tot = 0.5 * v2 - eps_iz;
                    const double e1 = u01(u[2]) * e_tot;
                    const double e2 = e_tot - e1;
                    const double g1 = sqrt(2.0 * e1), g2 = sqrt(2.0 * e2);
                    double d1[3], d2[3];
                    iso_dir(u1[0], u1[1], d1);
                    iso_dir(u1[2], u1[3], d2);
                    P->vx[p] = g1 * d1[0];
                    P->vy[p] = g1 * d1[1];
                    P->vz[p] = g1 * d1[2];
                    orc_iz_event *e = &ev[n_ev++];
                    e->parent = P->id[p];
                    e->x = P->x[p];
                    e->cell = (int64_t)floor(P->x[p]);
                    e->target = -1;
                    e->ve[0] = g2 * d2[0];
                    e->ve[1] = g2 * d2[1];
                    e->ve[2] = g2 * d2[2];
                    double n0, n1, n2, n3;
                    box_muller(u2[0], u2[1], &n0, &n1);
                    box_muller(u2[2], u2[3], &n2, &n3);
                    const double sig_i = sqrt(c->T_n / c->m[ki]) * (dt / dx);
                    e->vi[0] = sig_i * n0;
                    e->vi[1] = sig_i * n1;
                    e->vi[2] = sig_i * n2;
                    s->cnt.n_ionize++;
                }
            } else {
                if (r2 < C0 * v2) {
                    /* charge exchange: the ion takes a neutral's velocity */
                    uint32_t u1[4];
                    draw_block(c, P->id[p], step, 1, u1);
                    double n0, n1, n2, n3;
                    box_muller(u[2], u[3], &n0, &n1);
                    box_muller(u1[0], u1[1], &n2, &n3);
                    P->vx[p] = sig_n * n0;
                    P->vy[p] = sig_n * n1;
                    P->vz[p] = sig_n * n2;
                    s->cnt.n_cx++;
                }
            }
        }
        free(cand);
    }

    /* ids of created particles: events ordered by parent id; event r gives
     * the electron next_id + 2r and the ion next_id + 2r + 1 */
    if (n_ev > 1) qsort(ev, (size_t)n_ev, sizeof(orc_iz_event), cmp_event);
    /* the new electron stays at its parent; keep that position apart from
     * the ion's, which becomes the consumed atom's */
    double *xe = NULL;
    if (n_ev > 0) {
        xe = (double *)malloc(sizeof(double) * (size_t)n_ev);
        if (!xe) { free(ev); return -1; }
        for (int64_t r = 0; r < n_ev; ++r) xe[r] = ev[r].x;
    }
    if (kn >= 0 && n_ev > 0 && consume_neutrals(s, kn, ev, n_ev)) {
        free(xe);
        free(ev);
        return -1;
    }
    for (int64_t r = 0; r < n_ev; ++r) {
        append(s, ke, xe[r], ev[r].ve, s->cnt.next_id + 2 * (uint64_t)r);
        append(s, ki, ev[r].x, ev[r].vi, s->cnt.next_id + 2 * (uint64_t)r + 1);
    }
    s->cnt.next_id += 2 * (uint64_t)n_ev;
    free(xe);
    free(ev);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Volumetric pair source: as many electron-ion pairs as ions were absorbed   */
/* by the walls this step, each pair at one uniform position, velocities      */
/* Maxwellian at the species' source temperature.  Pair k takes the ids       */
/* next_id + 2k (electron) and next_id + 2k + 1 (ion).                        */
/* ------------------------------------------------------------------------ */
int orc_source(orc_sim *s)
{
    const orc_config *c = &s->cfg;
    if (!c->source_on) return 0;
    const int ke = find_kind(c, ORC_KIND_ELECTRON), ki = find_kind(c, ORC_KIND_ION);
    if (ke < 0 || ki < 0) return -1;
    const int64_t n_pairs = s->cnt.absorbed[ki][0] + s->cnt.absorbed[ki][1];
    const double dx = c->dx, dt = c->dt;
    const double se = sqrt(c->T_src[ke] / c->m[ke]) * (dt / dx);
    const double si = sqrt(c->T_src[ki] / c->m[ki]) * (dt / dx);
    const int64_t step = s->cnt.step;
    for (int64_t k = 0; k < n_pairs; ++k) {
        uint32_t b0[4], b1[4], b2[4];
        draw_block_source(c, (uint64_t)k, step, 0, b0);
        draw_block_source(c, (uint64_t)k, step, 1, b1);
        draw_block_source(c, (uint64_t)k, step, 2, b2);
        const double x = u01(b0[0]) * (double)c->nc;
        double e0, e1, e2, e3, i0, i1, i2, i3;
        box_muller(b0[1], b0[2], &e0, &e1);
        box_muller(b1[0], b1[1], &e2, &e3);
        box_muller(b1[2], b1[3], &i0, &i1);
        box_muller(b2[0], b2[1], &i2, &i3);
        double ve[3] = {se * e0, se * e1, se * e2};
        double vi[3] = {si * i0, si * i1, si * i2};
        append(s, ke, x, ve, s->cnt.next_id + 2 * (uint64_t)k);
        append(s, ki, x, vi, s->cnt.next_id + 2 * (uint64_t)k + 1);
    }
    s->cnt.next_id += 2 * (uint64_t)n_pairs;
    s->cnt.n_source += n_pairs;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One step: deposit(x^s) -> field -> push -> walls -> collisions -> source.  */
/* This is a rotation of the paper's cycle (density, smoother, field,         */
/* collisions/PWI, mover) with the smoother off; the collisions act on        */
/* v^{s+1/2} at x^{s+1} and use the step index s in their draws.              */
/* ------------------------------------------------------------------------ */
int orc_step(orc_sim *s)
{
    orc_deposit(s);
    if (orc_field(s)) return -1;
    orc_push(s);
    orc_walls(s);
    if (orc_mcc(s)) return -1;
    if (orc_source(s)) return -1;
    s->cnt.step++;
    return 0;
}

int orc_run(orc_sim *s, int64_t n_steps)
{
    for (int64_t i = 0; i < n_steps; ++i)
        if (orc_step(s)) return -1;
    return 0;
}

/* Diagnostics: per-species count, kinetic energy and momentum (SI, per unit
 * area), and the field energy of the last solve. */
void orc_diagnostics(const orc_sim *s, orc_diag *out)
{
    const orc_config *c = &s->cfg;
    memset(out, 0, sizeof(*out));
    const double vs = c->dx / c->dt;
    for (int k = 0; k < c->nsp; ++k) {
        const orc_particles *P = &s->sp[k];
        double s2 = 0.0, px = 0.0, py = 0.0, pz = 0.0;
        for (int64_t p = 0; p < P->n; ++p) {
            s2 += (P->vx[p] * P->vx[p] + P->vy[p] * P->vy[p]) + P->vz[p] * P->vz[p];
            px += P->vx[p];
            py += P->vy[p];
            pz += P->vz[p];
        }
        out->n[k] = P->n;
        out->ke[k] = 0.5 * c->m[k] * c->w[k] * (vs * vs) * s2;
        out->mom[k][0] = c->m[k] * c->w[k] * vs * px;
        out->mom[k][1] = c->m[k] * c->w[k] * vs * py;
        out->mom[k][2] = c->m[k] * c->w[k] * vs * pz;
    }
    double fe = 0.0;
    const int32_t nc = c->nc;
    if (c->bc == ORC_BC_PERIODIC) {
        for (int32_t j = 0; j < nc; ++j) fe += s->E[j] * s->E[j] * c->dx;
    } else {
        for (int32_t j = 0; j <= nc; ++j) {
            double V = (j == 0 || j == nc) ? 0.5 * c->dx : c->dx;
            fe += s->E[j] * s->E[j] * V;
        }
    }
    out->field_energy = 0.5 * c->eps0 * fe;
}

/* ------------------------------------------------------------------------ */
/* Initial particles drawn from the counter-based generator (the            */
/* configuration's own initial state, before step 0).  Particle p of        */
/* species k has id = (initial particles of the species before k) + p and   */
/* draws two Philox blocks at step -1:                                      */
/*   position  uniform x = U(u0) nc, or the lattice (p + 1/2) nc / n        */
/*             (quiet); with the pair option a species k > 0 of the same    */
/*             count as species 0 takes particle p of species 0's final     */
/*             position.  An electron species not so copied is displaced by */
/*             (A/kk) sin(kk x), kk = 2 pi m / nc (mode m, amplitude A),    */
/*             wrapped when periodic; every x is then kept inside [0, nc);  */
/*   velocity  Maxwellian, sqrt(T/m) dt/dx per component in cells/step:     */
/*             Box-Muller on (u1, u2) gives vx, vy; on (u3, u'0) gives vz.  */
/* This is the generator behind the X28 reading of the Langmuir start.      */
/* ------------------------------------------------------------------------ */
static double init_position(const orc_config *c, const int64_t *n_init, int k, int64_t p,
                            int quiet, double amp, int mode, uint64_t id)
{
    const int64_t n = n_init[k];
    const double L = (double)c->nc;
    double x;
    if (quiet) {
        x = ((double)p + 0.5) * L / (double)n;
    } else {
        uint32_t u[4];
        draw_block(c, id, -1, 0, u);
        x = u01(u[0]) * L;
    }
    if (amp != 0.0 && c->kind[k] == ORC_KIND_ELECTRON) {
        const double kk = 2.0 * M_PI * (double)mode / L;
        x = x + (amp / kk) * sin(kk * x);
        if (c->bc == ORC_BC_PERIODIC) x = x - L * floor(x / L);
    }
    if (x >= L) x = nextafter(L, 0.0);
    if (x < 0.0) x = 0.0;
    return x;
}

/* particle p of species k of the drawn initial state (see above) */
static void init_one(const orc_config *c, const int64_t *n_init, int k, int64_t p, int quiet,
                     int pair, double amp, int mode, double vth, double *x, double v[3],
                     uint64_t *id)
{
    int64_t id0 = 0;
    for (int q = 0; q < k; ++q) id0 += n_init[q];
    const uint64_t pid = (uint64_t)(id0 + p);
    const int copy = pair && k > 0 && n_init[k] == n_init[0];
    *id = pid;
    if (copy) *x = init_position(c, n_init, 0, p, quiet, amp, mode, (uint64_t)p);
    else *x = init_position(c, n_init, k, p, quiet, amp, mode, pid);
    uint32_t u[4], u1[4];
    draw_block(c, pid, -1, 0, u);
    draw_block(c, pid, -1, 1, u1);
    double n0, n1, n2, n3;
    box_muller(u[1], u[2], &n0, &n1);
    box_muller(u[3], u1[0], &n2, &n3);
    v[0] = vth * n0;
    v[1] = vth * n1;
    v[2] = vth * n2;
}

static double init_vth(const orc_config *c, int k, const double *T_init)
{
    return T_init[k] > 0.0 ? sqrt(T_init[k] / c->m[k]) * c->dt / c->dx : 0.0;
}

/* the particles p_list[0..m-1] of species k (all n_init[k] when p_list is NULL) */
void orc_init_species(const orc_config *c, const int64_t *n_init, int k, int quiet, int pair,
                      double amp, int mode, const double *T_init, int64_t m,
                      const int64_t *p_list, double *x, double *vx, double *vy, double *vz,
                      uint64_t *id)
{
    const double vth = init_vth(c, k, T_init);
    if (!p_list) m = n_init[k];
    for (int64_t q = 0; q < m; ++q) {
        const int64_t p = p_list ? p_list[q] : q;
        double v[3];
        init_one(c, n_init, k, p, quiet, pair, amp, mode, vth, &x[q], v, &id[q]);
        vx[q] = v[0];
        vy[q] = v[1];
        vz[q] = v[2];
    }
}

/* x as stored in the FP32 form: cell = floor(x), f = x - cell rounded to
 * float; an f that rounds to 1 moves to offset 0 of the next cell, or, in
 * the last cell, stays at the largest float below 1 */
double orc_fp32_form(double x, int32_t nc)
{
    double cell = floor(x);
    float f = (float)(x - cell);
    if (f >= 1.0f) {
        if (cell + 1.0 < (double)nc) {
            cell += 1.0;
            f = 0.0f;
        } else {
            f = nextafterf(1.0f, 0.0f);
        }
    }
    return cell + (double)f;
}

/* the fixed-point deposit of all n_init[k] drawn particles of species k,
 * computed particle by particle without storing them (S is cleared first);
 * with fp32 != 0 each position is first rounded to the FP32 storage form */
void orc_init_deposit(const orc_config *c, const int64_t *n_init, int k, int quiet, int pair,
                      double amp, int mode, int fp32, uint64_t *S)
{
    const int64_t n = n_init[k];
    const int copy = pair && k > 0 && n_init[k] == n_init[0];
    int64_t id0 = 0;
    for (int q = 0; q < k; ++q) id0 += n_init[q];
    memset(S, 0, sizeof(uint64_t) * (size_t)(c->nc + 1));
    for (int64_t p = 0; p < n; ++p) {
        double x = copy ? init_position(c, n_init, 0, p, quiet, amp, mode, (uint64_t)p)
                        : init_position(c, n_init, k, p, quiet, amp, mode, (uint64_t)(id0 + p));
        if (fp32) x = orc_fp32_form(x, c->nc);
        deposit_add(x, S);
    }
}

int orc_sizeof_sim(void) { return (int)sizeof(orc_sim); }
int orc_sizeof_config(void) { return (int)sizeof(orc_config); }
int orc_sizeof_counters(void) { return (int)sizeof(orc_counters); }
int orc_sizeof_diag(void) { return (int)sizeof(orc_diag); }

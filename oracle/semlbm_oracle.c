/*
 * Reference oracle for the two-phase spectral-element lattice Boltzmann time step
 * (Zhao, Patel & Lee, "Spectral element lattice Boltzmann method for non-ideal gases
 * with partial wetting boundary condition").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, FP64 CPU implementation that
 * the tests, the smoke check and the benchmark's CPU-baseline leg use to check the GPU
 * library.  Nothing in the product path may load it, and it shares no code with the
 * GPU library: the two are written separately from the paper.
 *
 * Every routine follows the paper's equations in the paper's order:
 *   - free energy and parameters: Appendix A, Eqs. (A.3)-(A.5)
 *   - chemical potential: Eq. (2) with its weak-form Laplacian, Eq. (8)
 *   - wetting condition: Eq. (7) and the normal-gradient relation of Sec. 2.2,
 *     entering only through the boundary integral of Eq. (8)
 *   - potential-form force and its split into F* and F**: Eq. (3) and Sec. 2.1
 *   - collision with modified distributions: Eq. (4), Eqs. (A.2), (A.6), (A.7)
 *   - weak-form streaming with force splitting: Eqs. (5), (6), (12)
 *   - flux bounce-back: Eq. (9)
 *   - third-order SSP Runge-Kutta time integration: Sec. 2.1
 *   - macroscopic moments: Eqs. (10), (11)
 *   - initial condition: Eqs. (A.1), (A.8), (A.9)
 *
 * Readings taken where the paper is silent or inconsistent (all listed in the design
 * notes of the repository):
 *   R1  continuous-Galerkin spectral elements (shared nodes, direct stiffness
 *       summation, GLL-lumped mass); the flux J acts on physical wall faces only.
 *   R3  mu0 = 2*beta*(rho-rl)*(rho-rv)*(2rho-rl-rv), the derivative of e0 of (A.3);
 *       Eq. (2) as printed lacks the factor 2.
 *   R4  streaming: d_t f + e.grad(f - t rho) + (t/cs^2) rho e.grad(mu) = 0, the sign
 *       that follows from F = cs^2 grad(rho) - rho grad(mu) and F* = (t/cs^2) e.F.
 *   R5  e.grad(f - t rho) is one derivative of the difference.
 *   R6  n is the outward normal of the fluid; n.grad(rho) = cos(theta) sqrt(2 e0/kappa).
 *   R7  sqrt(2 e0/kappa) = sqrt(2 beta/kappa) |(rho-rl)(rho-rv)|.
 *   R8  the pointwise collision uses the mass-weighted average of element gradients.
 *   R9  wall terms are evaluated per element face with that face's own normal.
 *   R10 rho, mu and their gradients are recomputed at every Runge-Kutta stage; stage 1
 *       uses the collision's rho and mu (collision conserves mass).
 *   R11 dt = min(CFL h_min, C h_min^2 / sqrt(kappa rho_l)) when no dt is given, C = 1/4
 *       for N <= 12 and 1/8 for N >= 13 (h_min: smallest distance between neighbouring GLL
 *       nodes along element lines; the second bound is the capillary stiffness limit of the
 *       force term).
 *   R12 tau is dimensionless: omega = 1/(tau + 1/2), and the kinematic viscosity is
 *       tau cs^2 dt; given a viscosity nu > 0, tau = 3 nu / dt.
 *   R16 seeded density noise: rho += a (2U - 1), U from SplitMix64 of (seed xor gid).
 *
 * Threads: the element loops and the pointwise node loops may run on several host
 * threads (OpenMP, orc_set_threads; one thread unless set).  Their iterations write
 * disjoint entries, and every sum over nodes (the direct stiffness summation, the mass)
 * stays a sequential loop, so the results do not depend on the thread count.
 *
 * Arithmetic conventions (so that a separately written implementation can follow the
 * same expression trees): sums run in ascending index order starting from 0; the
 * tensor-product contractions with the GLL differentiation matrix use fused
 * multiply-add, every other operation is a plain IEEE operation; this file must be
 * compiled without floating-point contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OQ_MAX 19

typedef struct {
    int dim, N, Np, nloc, Q, mode;
    long E, Nl, Ng;
    /* lattice (Appendix-A tables) */
    double ev[OQ_MAX][3];
    double tw[OQ_MAX];
    int opp[OQ_MAX];
    /* GLL */
    double *xi, *w, *D; /* D[i*Np+m] = l_m'(xi_i) */
    double *wn;         /* [nloc] tensor weight products */
    /* mesh */
    int *gid;    /* [Nl] */
    double *xyz; /* [Nl*dim] */
    /* geometry */
    double *Ja;  /* [Nl*9]  Ja[a][c] = J d xi_a / d x_c at [l*9 + a*3 + c] */
    double *Jac; /* [Nl] */
    double *G;   /* [Nl*9] */
    double *MA, *Minv;
    /* wall entries: one per (wall face, face node) */
    long nw;
    long *wl;     /* local node */
    double *wsn;  /* [nw*3] s*n */
    double *ws;   /* [nw] s */
    double *wcos; /* [nw] */
    double *wub;  /* [nw*3] */
    /* parameters */
    double rho_l, rho_v, delta, sigma, tau, dt, cfl, nu, beta, kappa, omega, hmin;
    /* state */
    double *f; /* [Q*Ng] */
    long nstep;
    /* scratch */
    double *rl;  /* [Q*Nl] */
    double *tmp; /* [Q*Ng] */
} orc;

/* host threads of the parallel loops (1 by default, see the header note) */
void orc_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* GLL nodes, weights and differentiation matrix (Deville, Fischer & Mund, ch. 2)       */
/* ------------------------------------------------------------------------------------ */

static void legendre(int N, double x, double *P, double *dP) {
    /* Bonnet recurrence for P_N and its derivative */
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (N == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *P = p1; *dP = d1;
}

static void gll(int N, double *x, double *w, double *D) {
    int Np = N + 1;
    x[0] = -1.0; x[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double t = -cos(M_PI * i / N); /* Chebyshev-Gauss-Lobatto start */
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(N, t, &P, &dP);
            /* Legendre ODE: (1-x^2) P'' = 2x P' - N(N+1) P */
            double d2P = (2.0 * t * dP - N * (N + 1.0) * P) / (1.0 - t * t);
            double dx = dP / d2P;
            t -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        x[i] = t;
    }
    for (int i = 0; i < Np / 2; ++i) { /* exact symmetry */
        double s = 0.5 * (x[N - i] - x[i]);
        x[N - i] = s; x[i] = -s;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
    double PN[64];
    for (int i = 0; i < Np; ++i) {
        double dP;
        legendre(N, x[i], &PN[i], &dP);
        w[i] = 2.0 / (N * (N + 1.0) * PN[i] * PN[i]);
    }
    for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Np; ++j) {
            double v;
            if (i != j) v = PN[i] / (PN[j] * (x[i] - x[j]));
            else if (i == 0) v = -N * (N + 1.0) / 4.0;
            else if (i == N) v = N * (N + 1.0) / 4.0;
            else v = 0.0;
            D[i * Np + j] = v;
        }
}

/* ------------------------------------------------------------------------------------ */
/* lattices: D2Q9 (Sec. 2.1), D3Q19 and D3Q13                                        */
/* ------------------------------------------------------------------------------------ */

static int set_lattice(orc *o, int Q) {
    memset(o->ev, 0, sizeof o->ev);
    if (Q == 9) {
        static const int E9[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                     {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
        for (int a = 0; a < 9; ++a) {
            o->ev[a][0] = E9[a][0]; o->ev[a][1] = E9[a][1];
            o->tw[a] = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
    } else if (Q == 19) {
        static const int E19[19][3] = {
            {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
            {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
            {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        for (int a = 0; a < 19; ++a) {
            for (int c = 0; c < 3; ++c) o->ev[a][c] = E19[a][c];
            o->tw[a] = a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
    } else if (Q == 13) {
        /* 13 velocities in 3-D (Sec. 3.2 uses a 13-velocity model), reading R22.  With a
         * rest weight t0 and one weight t1 for twelve moving velocities of speed |e|, the
         * equilibrium (A.2) has the moments rho, rho u and rho cs^2 I + rho u u only if
         *   sum t = 1, sum t e_i e_j = cs^2 d_ij, sum t e_i e_j e_k = 0 and
         *   sum t e_i e_j e_k e_l = cs^4 (d_ij d_kl + d_ik d_jl + d_il d_jk).
         * The twelve face diagonals of a cube (the cubic 13-velocity set) give
         * sum e_x^4 = 2 sum e_x^2 e_y^2 and cannot meet the last condition; the twelve
         * vertices of an icosahedron, a spherical 5-design, give
         *   sum e_i e_j = 4 |e|^2 d_ij and sum e_i e_j e_k e_l = (4/5)|e|^4 (d d + d d + d d),
         * so 4 |e|^2 t1 = cs^2 and (4/5)|e|^4 t1 = cs^4: |e|^2 = 5 cs^2 = 5/3, t1 = 1/20 and
         * t0 = 2/5.  The vertices (0, +-1, +-phi) and their cyclic permutations, scaled to
         * |e|^2 = 5/3, have components of magnitude
         *   a = sqrt((5 - sqrt 5) / 6) and b = phi a = sqrt((5 + sqrt 5) / 6).
         * Population order (1 = a, 2 = b, signs as written): opposite pairs are adjacent. */
        static const int P13[13][3] = {{0, 0, 0},  {0, 1, 2},   {0, -1, -2}, {0, 1, -2}, {0, -1, 2},
                                       {1, 2, 0},  {-1, -2, 0}, {1, -2, 0},  {-1, 2, 0}, {2, 0, 1},
                                       {-2, 0, -1}, {2, 0, -1}, {-2, 0, 1}};
        double ma = sqrt((5.0 - sqrt(5.0)) / 6.0), mb = sqrt((5.0 + sqrt(5.0)) / 6.0);
        for (int a = 0; a < 13; ++a) {
            for (int c = 0; c < 3; ++c) {
                int k = P13[a][c];
                double m = (k == 1 || k == -1) ? ma : mb;
                o->ev[a][c] = k == 0 ? 0.0 : (k > 0 ? m : -m);
            }
            o->tw[a] = a == 0 ? 2.0 / 5.0 : 1.0 / 20.0;
        }
    } else
        return -1;
    /* The rest weight is chosen so that the FP64 weights sum to exactly one: it is
     * 1 minus the exact sum of the moving weights (error-free TwoSum accumulation,
     * Knuth), which is representable for both lattices.  With the nearest double of
     * 4/9 (1/3) the weights would sum to 1 - 5.6e-17 (1 - 2.2e-16) and every
     * collision would bleed that fraction of the mass. */
    {
        double s = 0.0, err = 0.0;
        for (int a = 1; a < Q; ++a) {
            double t = s + o->tw[a];
            double bp = t - s;
            err += (s - (t - bp)) + (o->tw[a] - bp);
            s = t;
        }
        o->tw[0] = (1.0 - s) - err;
    }
    o->Q = Q;
    for (int a = 0; a < Q; ++a) {
        o->opp[a] = -1;
        for (int b = 0; b < Q; ++b)
            if (o->ev[b][0] == -o->ev[a][0] && o->ev[b][1] == -o->ev[a][1] &&
                o->ev[b][2] == -o->ev[a][2])
                o->opp[a] = b;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* tensor-product derivative along reference direction a at local node n                */
/* ------------------------------------------------------------------------------------ */

static int stride_of(const orc *o, int a) { return a == 0 ? 1 : (a == 1 ? o->Np : o->Np * o->Np); }
static int idx_along(const orc *o, int n, int a) { return (n / stride_of(o, a)) % o->Np; }

/* (D h)_a at n: sum_m D[i_a][m] h[n with i_a = m] */
static double dref(const orc *o, const double *h, int n, int a) {
    int s = stride_of(o, a), i = idx_along(o, n, a), base = n - i * s;
    double acc = 0.0;
    for (int m = 0; m < o->Np; ++m) acc = fma(o->D[i * o->Np + m], h[base + m * s], acc);
    return acc;
}

/* (D^T v)_a at n: sum_m D[m][i_a] v[n with i_a = m] */
static double drefT(const orc *o, const double *v, int n, int a) {
    int s = stride_of(o, a), i = idx_along(o, n, a), base = n - i * s;
    double acc = 0.0;
    for (int m = 0; m < o->Np; ++m) acc = fma(o->D[m * o->Np + i], v[base + m * s], acc);
    return acc;
}

/* ------------------------------------------------------------------------------------ */
/* construction                                                                         */
/* ------------------------------------------------------------------------------------ */

void orc_free(orc *o);

/* phys = {rho_l, rho_v, delta, sigma, tau, dt, cfl, nu}; nu > 0 replaces tau by the
 * relaxation time of that kinematic viscosity at the time step (R12); mode 0 = two-phase step,
 * mode 1 = pure advection of every population (no force, no collision). */
orc *orc_new(int dim, int N, int Q, long E, const double *xyz, const int *gid, long ng,
             long nwf, const int *wf, const double *wcos, const double *wub,
             const double *phys, int mode) {
    if ((dim != 2 && dim != 3) || N < 1 || N > 32 || E < 1) return NULL;
    orc *o = (orc *)calloc(1, sizeof(orc));
    o->dim = dim; o->N = N; o->Np = N + 1; o->mode = mode;
    o->nloc = dim == 2 ? o->Np * o->Np : o->Np * o->Np * o->Np;
    if (o->nloc > 4096) { free(o); return NULL; } /* element scratch arrays below */
    o->E = E; o->Nl = E * o->nloc; o->Ng = ng;
    if (set_lattice(o, Q) || (Q == 9) != (dim == 2)) { free(o); return NULL; }
    o->xi = malloc(sizeof(double) * o->Np);
    o->w = malloc(sizeof(double) * o->Np);
    o->D = malloc(sizeof(double) * o->Np * o->Np);
    gll(N, o->xi, o->w, o->D);
    o->wn = malloc(sizeof(double) * o->nloc);
    for (int n = 0; n < o->nloc; ++n) {
        double p = o->w[idx_along(o, n, 0)] * o->w[idx_along(o, n, 1)];
        if (dim == 3) p = p * o->w[idx_along(o, n, 2)];
        o->wn[n] = p;
    }
    o->gid = malloc(sizeof(int) * o->Nl);
    memcpy(o->gid, gid, sizeof(int) * o->Nl);
    o->xyz = malloc(sizeof(double) * o->Nl * dim);
    memcpy(o->xyz, xyz, sizeof(double) * o->Nl * dim);
    o->rho_l = phys[0]; o->rho_v = phys[1]; o->delta = phys[2]; o->sigma = phys[3];
    o->tau = phys[4]; o->dt = phys[5]; o->cfl = phys[6]; o->nu = phys[7];
    /* (A.4)-(A.5) solved for beta, kappa at gamma = sigma */
    double dr = o->rho_l - o->rho_v;
    o->beta = 12.0 * o->sigma / (o->delta * dr * dr * dr * dr);
    o->kappa = 3.0 * o->sigma * o->delta / (2.0 * dr * dr);
    o->omega = 1.0 / (o->tau + 0.5);

    long Nl = o->Nl;
    o->Ja = calloc(Nl * 9, sizeof(double));
    o->Jac = calloc(Nl, sizeof(double));
    o->G = calloc(Nl * 9, sizeof(double));
    o->MA = calloc(ng, sizeof(double));
    o->Minv = calloc(ng, sizeof(double));
    int nloc = o->nloc;
    double *X = malloc(sizeof(double) * 3 * nloc);
    double *dX = malloc(sizeof(double) * 9 * nloc); /* dX[(c*3+a)*nloc + n] = d x_c / d xi_a */
    double *V = malloc(sizeof(double) * 3 * nloc);
    o->hmin = INFINITY;
    for (long e = 0; e < E; ++e) {
        for (int n = 0; n < nloc; ++n)
            for (int c = 0; c < dim; ++c) X[c * nloc + n] = xyz[(e * nloc + n) * dim + c];
        for (int c = 0; c < dim; ++c)
            for (int a = 0; a < dim; ++a)
                for (int n = 0; n < nloc; ++n)
                    dX[(c * 3 + a) * nloc + n] = dref(o, X + c * nloc, n, a);
        double *Ja = o->Ja + e * nloc * 9;
        if (dim == 2) {
            for (int n = 0; n < nloc; ++n) {
                double xa = dX[0 * nloc + n], xb = dX[1 * nloc + n];      /* x_xi, x_eta */
                double ya = dX[3 * nloc + n], yb = dX[4 * nloc + n];      /* y_xi, y_eta */
                double *J = Ja + n * 9;
                J[0 * 3 + 0] = yb;  J[0 * 3 + 1] = -xb;  /* J grad(xi)  = (y_eta, -x_eta) */
                J[1 * 3 + 0] = -ya; J[1 * 3 + 1] = xa;   /* J grad(eta) = (-y_xi, x_xi) */
                o->Jac[e * nloc + n] = xa * yb - xb * ya;
            }
        } else {
            /* Kopriva's conservative curl form: J grad(xi_i)_n = -[curl_xi (x_l grad_xi x_m)]_i
             * with (n, m, l) cyclic, so the discrete metric identities hold exactly. */
            for (int cn = 0; cn < 3; ++cn) {
                int cm = (cn + 1) % 3, cl = (cn + 2) % 3;
                for (int k = 0; k < 3; ++k)
                    for (int n = 0; n < nloc; ++n)
                        V[k * nloc + n] = X[cl * nloc + n] * dX[(cm * 3 + k) * nloc + n];
                for (int n = 0; n < nloc; ++n) {
                    double c0 = dref(o, V + 2 * nloc, n, 1) - dref(o, V + 1 * nloc, n, 2);
                    double c1 = dref(o, V + 0 * nloc, n, 2) - dref(o, V + 2 * nloc, n, 0);
                    double c2 = dref(o, V + 1 * nloc, n, 0) - dref(o, V + 0 * nloc, n, 1);
                    Ja[n * 9 + 0 * 3 + cn] = -c0;
                    Ja[n * 9 + 1 * 3 + cn] = -c1;
                    Ja[n * 9 + 2 * 3 + cn] = -c2;
                }
            }
            for (int n = 0; n < nloc; ++n) {
                double a0 = dX[0 * nloc + n], a1 = dX[3 * nloc + n], a2 = dX[6 * nloc + n]; /* x_xi */
                double b0 = dX[1 * nloc + n], b1 = dX[4 * nloc + n], b2 = dX[7 * nloc + n]; /* x_eta */
                double c0 = dX[2 * nloc + n], c1 = dX[5 * nloc + n], c2 = dX[8 * nloc + n]; /* x_zeta */
                double cx = b1 * c2 - b2 * c1, cy = b2 * c0 - b0 * c2, cz = b0 * c1 - b1 * c0;
                o->Jac[e * nloc + n] = a0 * cx + a1 * cy + a2 * cz;
            }
        }
        for (int n = 0; n < nloc; ++n) {
            long l = e * nloc + n;
            double J = o->Jac[l];
            if (!(J > 0.0)) { free(X); free(dX); free(V); orc_free(o); return NULL; }
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < dim; ++b) {
                    double s = 0.0;
                    for (int c = 0; c < dim; ++c) s += Ja[n * 9 + a * 3 + c] * Ja[n * 9 + b * 3 + c];
                    o->G[l * 9 + a * 3 + b] = o->wn[n] * s / J;
                }
            o->MA[gid[l]] += o->wn[n] * J;
        }
        /* smallest neighbour distance along element lines (R11) */
        for (int a = 0; a < dim; ++a) {
            int s = stride_of(o, a);
            for (int n = 0; n < nloc; ++n) {
                if (idx_along(o, n, a) == o->N) continue;
                double d2 = 0.0;
                for (int c = 0; c < dim; ++c) {
                    double dd = X[c * nloc + n + s] - X[c * nloc + n];
                    d2 += dd * dd;
                }
                double d = sqrt(d2);
                if (d < o->hmin) o->hmin = d;
            }
        }
    }
    free(X); free(dX); free(V);
    for (long g = 0; g < ng; ++g) o->Minv[g] = 1.0 / o->MA[g];
    if (!(o->dt > 0.0)) {
        /* advective limit, and the capillary limit of the kappa lap(rho) term inside the
         * streaming force, whose discrete spectrum grows like h^-2 (stable dt ~ h^2); the
         * capillary constant is 1/4 up to order 12 and 1/8 above (R11) */
        double dt_adv = o->cfl * o->hmin;
        double c_cap = o->N > 12 ? 0.125 : 0.25;
        double dt_cap = c_cap * o->hmin * o->hmin / sqrt(o->kappa * o->rho_l);
        o->dt = dt_adv < dt_cap ? dt_adv : dt_cap;
    }
    if (o->nu > 0.0) {
        /* R12: the kinematic viscosity is tau cs^2 dt with cs^2 = 1/3 */
        o->tau = 3.0 * o->nu / o->dt;
        o->omega = 1.0 / (o->tau + 0.5);
    }

    /* wall entries, in the order of the face list, face nodes ascending (R9) */
    int nfn = dim == 2 ? o->Np : o->Np * o->Np;
    o->nw = nwf * nfn;
    o->wl = malloc(sizeof(long) * (o->nw + 1));
    o->wsn = calloc(o->nw * 3 + 1, sizeof(double));
    o->ws = calloc(o->nw + 1, sizeof(double));
    o->wcos = calloc(o->nw + 1, sizeof(double));
    o->wub = calloc(o->nw * 3 + 1, sizeof(double));
    long k = 0;
    for (long fidx = 0; fidx < nwf; ++fidx) {
        long e = wf[2 * fidx];
        int face = wf[2 * fidx + 1], a = face / 2, side = face % 2;
        double sign = side ? 1.0 : -1.0;
        for (int n = 0; n < nloc; ++n) {
            if (idx_along(o, n, a) != (side ? o->N : 0)) continue;
            double wf_ = 1.0;
            for (int b = 0; b < dim; ++b)
                if (b != a) wf_ = wf_ * o->w[idx_along(o, n, b)];
            long l = e * nloc + n;
            const double *J = o->Ja + l * 9 + a * 3;
            double nrm2 = 0.0;
            for (int c = 0; c < dim; ++c) nrm2 += J[c] * J[c];
            o->wl[k] = l;
            for (int c = 0; c < dim; ++c) o->wsn[k * 3 + c] = sign * wf_ * J[c];
            o->ws[k] = wf_ * sqrt(nrm2);
            o->wcos[k] = wcos[fidx];
            for (int c = 0; c < dim; ++c) o->wub[k * 3 + c] = wub ? wub[fidx * dim + c] : 0.0;
            ++k;
        }
    }
    o->f = calloc((size_t)Q * ng, sizeof(double));
    o->rl = calloc((size_t)Q * Nl, sizeof(double));
    o->tmp = calloc((size_t)Q * ng, sizeof(double));
    return o;
}

void orc_free(orc *o) {
    if (!o) return;
    free(o->xi); free(o->w); free(o->D); free(o->wn); free(o->gid); free(o->xyz);
    free(o->Ja); free(o->Jac); free(o->G); free(o->MA); free(o->Minv);
    free(o->wl); free(o->wsn); free(o->ws); free(o->wcos); free(o->wub);
    free(o->f); free(o->rl); free(o->tmp);
    free(o);
}

/* info: dt, beta, kappa, omega, hmin, Ng, Nl, nw */
void orc_info(const orc *o, double *out) {
    out[0] = o->dt; out[1] = o->beta; out[2] = o->kappa; out[3] = o->omega; out[4] = o->hmin;
    out[5] = (double)o->Ng; out[6] = (double)o->Nl; out[7] = (double)o->nw;
}

void orc_gll(const orc *o, double *x, double *w, double *D) {
    memcpy(x, o->xi, sizeof(double) * o->Np);
    memcpy(w, o->w, sizeof(double) * o->Np);
    memcpy(D, o->D, sizeof(double) * o->Np * o->Np);
}

void orc_lattice(const orc *o, double *ev, double *tw, int *opp) {
    for (int a = 0; a < o->Q; ++a) {
        for (int c = 0; c < 3; ++c) ev[a * 3 + c] = o->ev[a][c];
        tw[a] = o->tw[a];
        opp[a] = o->opp[a];
    }
}

void orc_mass_matrix(const orc *o, double *MA) { memcpy(MA, o->MA, sizeof(double) * o->Ng); }

/* wall entries: local node, s*n[3], s */
void orc_wall_entries(const orc *o, long *wl, double *wsn, double *ws) {
    memcpy(wl, o->wl, sizeof(long) * o->nw);
    memcpy(wsn, o->wsn, sizeof(double) * 3 * o->nw);
    memcpy(ws, o->ws, sizeof(double) * o->nw);
}

/* ------------------------------------------------------------------------------------ */
/* direct stiffness summation and operators                                             */
/* ------------------------------------------------------------------------------------ */

/* R[g] = sum over local copies (ascending local index) of r[l] */
static void dss(const orc *o, const double *r, double *R) {
    memset(R, 0, sizeof(double) * o->Ng);
    for (long l = 0; l < o->Nl; ++l) R[o->gid[l]] += r[l];
}

/* weak Laplacian, Eq. (8): lap = M^-1 ( sum_wall s n.grad(rho) - K rho ), with the
 * wetting normal gradient (Sec. 2.2) when with_wall != 0 */
void orc_lap(orc *o, const double *rho, double *lap, int with_wall) {
    int nloc = o->nloc, dim = o->dim;
    double *r = o->rl;
    double sq = sqrt(2.0 * o->beta / o->kappa);
#pragma omp parallel for schedule(static)
    for (long e = 0; e < o->E; ++e) {
        double re[4096], d[3][4096], v[3][4096];
        for (int n = 0; n < nloc; ++n) re[n] = rho[o->gid[e * nloc + n]];
        for (int a = 0; a < dim; ++a)
            for (int n = 0; n < nloc; ++n) d[a][n] = dref(o, re, n, a);
        for (int n = 0; n < nloc; ++n) {
            const double *G = o->G + (e * nloc + n) * 9;
            for (int a = 0; a < dim; ++a) {
                double s = 0.0;
                for (int b = 0; b < dim; ++b) s += G[a * 3 + b] * d[b][n];
                v[a][n] = s;
            }
        }
        for (int n = 0; n < nloc; ++n) {
            double s = 0.0;
            for (int a = 0; a < dim; ++a) s += drefT(o, v[a], n, a);
            r[e * nloc + n] = -s;
        }
    }
    if (with_wall)
        for (long k = 0; k < o->nw; ++k) {
            long l = o->wl[k];
            double rh = rho[o->gid[l]];
            double wsc = o->ws[k] * o->wcos[k] * sq;
            r[l] += wsc * fabs((rh - o->rho_l) * (rh - o->rho_v));
        }
    dss(o, r, lap);
#pragma omp parallel for schedule(static)
    for (long g = 0; g < o->Ng; ++g) lap[g] = lap[g] * o->Minv[g];
}

/* chemical potential, Eq. (2) with reading R3 */
void orc_mu(orc *o, const double *rho, double *mu) {
    orc_lap(o, rho, mu, 1);
    double rl = o->rho_l, rv = o->rho_v;
#pragma omp parallel for schedule(static)
    for (long g = 0; g < o->Ng; ++g) {
        double p = rho[g];
        double mu0 = 2.0 * o->beta * (p - rl) * (p - rv) * (2.0 * p - rl - rv);
        mu[g] = mu0 - o->kappa * mu[g];
    }
}

/* mass-weighted average of element gradients (R8): grad[c*Ng + g] */
void orc_avg_grad(orc *o, const double *phi, double *grad) {
    int nloc = o->nloc, dim = o->dim;
    for (int c = 0; c < dim; ++c) {
#pragma omp parallel for schedule(static)
        for (long e = 0; e < o->E; ++e) {
            double pe[4096], d[3][4096];
            for (int n = 0; n < nloc; ++n) pe[n] = phi[o->gid[e * nloc + n]];
            for (int a = 0; a < dim; ++a)
                for (int n = 0; n < nloc; ++n) d[a][n] = dref(o, pe, n, a);
            for (int n = 0; n < nloc; ++n) {
                const double *Ja = o->Ja + (e * nloc + n) * 9;
                double s = 0.0;
                for (int a = 0; a < dim; ++a) s += Ja[a * 3 + c] * d[a][n];
                o->rl[e * nloc + n] = o->wn[n] * s;
            }
        }
        dss(o, o->rl, grad + c * o->Ng);
#pragma omp parallel for schedule(static)
        for (long g = 0; g < o->Ng; ++g) grad[c * o->Ng + g] = grad[c * o->Ng + g] * o->Minv[g];
    }
}

/* streaming operator of Eqs. (5), (6), (12) with flux bounce-back, Eq. (9):
 * L[a*Ng + g] = M^-1 DSS( B[-e.grad(g_a - t_a rho) - (t_a/cs^2) rho e.grad(mu)] + J terms ) */
void orc_stream_op(orc *o, const double *g, const double *rho, const double *mu, double *L) {
    int nloc = o->nloc, dim = o->dim, Q = o->Q;
    long Ng = o->Ng, Nl = o->Nl;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < o->E; ++e) {
        double he[4096], me[4096], dh[3][4096], dm[3][4096];
        const int *gd = o->gid + e * nloc;
        if (o->mode == 0) {
            for (int n = 0; n < nloc; ++n) me[n] = mu[gd[n]];
            for (int a = 0; a < dim; ++a)
                for (int n = 0; n < nloc; ++n) dm[a][n] = dref(o, me, n, a);
        }
        for (int q = 1; q < Q; ++q) {
            double tq = o->tw[q], tc = 3.0 * tq;
            for (int n = 0; n < nloc; ++n)
                he[n] = o->mode == 0 ? g[q * Ng + gd[n]] - tq * rho[gd[n]] : g[q * Ng + gd[n]];
            for (int a = 0; a < dim; ++a)
                for (int n = 0; n < nloc; ++n) dh[a][n] = dref(o, he, n, a);
            for (int n = 0; n < nloc; ++n) {
                const double *Ja = o->Ja + (e * nloc + n) * 9;
                double adv = 0.0, frc = 0.0;
                for (int a = 0; a < dim; ++a) {
                    double ca = 0.0;
                    for (int c = 0; c < dim; ++c) ca += Ja[a * 3 + c] * o->ev[q][c];
                    adv += ca * dh[a][n];
                    if (o->mode == 0) frc += ca * dm[a][n];
                }
                double r;
                if (o->mode == 0) r = -(o->wn[n] * (adv + tc * rho[gd[n]] * frc));
                else r = -(o->wn[n] * adv);
                o->rl[(size_t)q * Nl + e * nloc + n] = r;
            }
        }
    }
    for (long k = 0; k < o->nw; ++k) {
        long l = o->wl[k];
        int gg = o->gid[l];
        for (int q = 1; q < Q; ++q) {
            double cn = 0.0;
            for (int c = 0; c < dim; ++c) cn += o->wsn[k * 3 + c] * o->ev[q][c];
            if (!(cn < 0.0)) continue; /* incoming populations only */
            double eub = 0.0;
            for (int c = 0; c < dim; ++c) eub += o->ev[q][c] * o->wub[k * 3 + c];
            double tc = 3.0 * o->tw[q];
            double bc = g[q * Ng + gg] - g[o->opp[q] * Ng + gg] - 2.0 * tc * rho[gg] * eub;
            o->rl[(size_t)q * Nl + l] += cn * bc;
        }
    }
    memset(L, 0, sizeof(double) * Ng); /* rest population does not stream */
    for (int q = 1; q < Q; ++q) {
        dss(o, o->rl + (size_t)q * Nl, L + q * Ng);
#pragma omp parallel for schedule(static)
        for (long gg = 0; gg < Ng; ++gg) L[q * Ng + gg] = L[q * Ng + gg] * o->Minv[gg];
    }
}

/* density, Eq. (10) */
void orc_density(const orc *o, const double *f, double *rho) {
#pragma omp parallel for schedule(static)
    for (long g = 0; g < o->Ng; ++g) {
        double s = 0.0;
        for (int q = 0; q < o->Q; ++q) s += f[q * o->Ng + g];
        rho[g] = s;
    }
}

/* collision, Eq. (4) with the modified distributions (A.6)-(A.7), the higher-order force
 * F** of Sec. 2.1 and the equilibrium (A.2); F = cs^2 grad(rho) - rho grad(mu), Eq. (3) */
void orc_collide(const orc *o, const double *f, const double *rho, const double *grho,
                 const double *gmu, double *fs) {
    int dim = o->dim, Q = o->Q;
    long Ng = o->Ng;
    double cs2 = 1.0 / 3.0, dt = o->dt, om = o->omega;
#pragma omp parallel for schedule(static)
    for (long g = 0; g < Ng; ++g) {
        double p = rho[g], u[3] = {0, 0, 0}, F[3] = {0, 0, 0};
        for (int c = 0; c < dim; ++c) {
            double m = 0.0;
            for (int q = 0; q < Q; ++q) m += f[q * Ng + g] * o->ev[q][c];
            u[c] = m / p;
            F[c] = cs2 * grho[c * Ng + g] - p * gmu[c * Ng + g];
        }
        double uF = 0.0, uu = 0.0;
        for (int c = 0; c < dim; ++c) { uF += u[c] * F[c]; uu += u[c] * u[c]; }
        for (int q = 0; q < Q; ++q) {
            double eu = 0.0, eF = 0.0;
            for (int c = 0; c < dim; ++c) { eu += o->ev[q][c] * u[c]; eF += o->ev[q][c] * F[c]; }
            double tq = o->tw[q], tc = 3.0 * tq;
            double Fss = tc * (eu * eF * 3.0 - uF);
            double feq = p * tq * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
            double fbeq = feq - 0.5 * dt * Fss;
            double fq = f[q * Ng + g];
            fs[q * Ng + g] = fq - om * (fq - fbeq) + dt * Fss;
        }
    }
}

/* SSP-RK3 stage combinations (Shu-Osher form):
 *   stage 1: g1 = g0 + dt L
 *   stage 2: g2 = 3/4 g0 + 1/4 (g1 + dt L)
 *   stage 3: f  = (g0 + 2 (g2 + dt L)) / 3   -- written with one division so that the
 *            two weights do not sum to fl(1/3) + fl(2/3) < 1 */
static void rk_combine(const orc *o, int stage, const double *g0, const double *g,
                       const double *L, double *gout) {
    long n = (long)o->Q * o->Ng;
    double dt = o->dt;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double x = g[i] + dt * L[i];
        if (stage == 1) gout[i] = x;
        else if (stage == 2) gout[i] = 0.75 * g0[i] + 0.25 * x;
        else gout[i] = (g0[i] + 2.0 * x) / 3.0;
    }
}

/* one time step: collision, then three SSP-RK3 streaming stages (Sec. 2.1) */
void orc_step(orc *o, long nsteps) {
    long Ng = o->Ng, QN = (long)o->Q * Ng;
    int dim = o->dim;
    double *rho = malloc(sizeof(double) * Ng), *mu = malloc(sizeof(double) * Ng);
    double *gr = malloc(sizeof(double) * dim * Ng), *gm = malloc(sizeof(double) * dim * Ng);
    double *g0 = malloc(sizeof(double) * QN), *g1 = malloc(sizeof(double) * QN);
    double *L = malloc(sizeof(double) * QN);
    for (long s = 0; s < nsteps; ++s) {
        orc_density(o, o->f, rho);
        if (o->mode == 0) {
            orc_mu(o, rho, mu);
            orc_avg_grad(o, rho, gr);
            orc_avg_grad(o, mu, gm);
            orc_collide(o, o->f, rho, gr, gm, g0);
        } else {
            memcpy(g0, o->f, sizeof(double) * QN);
        }
        /* stage 1: g1 = g0 + dt L(g0), with the collision's rho and mu (R10) */
        orc_stream_op(o, g0, rho, mu, L);
        rk_combine(o, 1, g0, g0, L, g1);
        /* stage 2: g2 = 3/4 g0 + 1/4 (g1 + dt L(g1)) */
        orc_density(o, g1, rho);
        if (o->mode == 0) orc_mu(o, rho, mu);
        orc_stream_op(o, g1, rho, mu, L);
        rk_combine(o, 2, g0, g1, L, g1);
        /* stage 3: f = 1/3 g0 + 2/3 (g2 + dt L(g2)) */
        orc_density(o, g1, rho);
        if (o->mode == 0) orc_mu(o, rho, mu);
        orc_stream_op(o, g1, rho, mu, L);
        rk_combine(o, 3, g0, g1, L, o->f);
        o->nstep++;
    }
    free(rho); free(mu); free(gr); free(gm); free(g0); free(g1); free(L);
}

/* ------------------------------------------------------------------------------------ */
/* state, initial condition and queries                                                 */
/* ------------------------------------------------------------------------------------ */

/* f = t_a rho, u = 0: equilibrium with F** = 0 */
void orc_set_rho(orc *o, const double *rho) {
    for (int q = 0; q < o->Q; ++q)
        for (long g = 0; g < o->Ng; ++g) o->f[q * o->Ng + g] = o->tw[q] * rho[g];
}

void orc_set_f(orc *o, const double *f) { memcpy(o->f, f, sizeof(double) * o->Q * o->Ng); }
void orc_get_f(const orc *o, double *f) { memcpy(f, o->f, sizeof(double) * o->Q * o->Ng); }
long orc_nstep(const orc *o) { return o->nstep; }

/* SplitMix64 (Steele, Lea & Flood 2014): one output from state x */
static uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t x) { return splitmix64(x); }

/* Eqs. (A.1)/(A.8)-(A.9): tanh profile of the signed distance |x - x0| - R (liquid
 * inside), coordinates of a global node taken from its lowest local copy, plus
 * seeded noise a(2U-1) per global id (R16) */
void orc_init_tanh(orc *o, const double *x0, double R, double amp, uint64_t seed) {
    long Ng = o->Ng;
    int dim = o->dim;
    double *rho = malloc(sizeof(double) * Ng);
    char *done = calloc(Ng, 1);
    for (long l = 0; l < o->Nl; ++l) {
        int g = o->gid[l];
        if (done[g]) continue;
        done[g] = 1;
        double r2 = 0.0;
        for (int c = 0; c < dim; ++c) {
            double d = o->xyz[l * dim + c] - x0[c];
            r2 += d * d;
        }
        double x = sqrt(r2) - R;
        double p = 0.5 * (o->rho_l + o->rho_v) - 0.5 * (o->rho_l - o->rho_v) * tanh(2.0 * x / o->delta);
        if (amp != 0.0) {
            uint64_t h = splitmix64(seed ^ (uint64_t)g);
            double U = (double)(h >> 11) * 0x1.0p-53;
            p += amp * (2.0 * U - 1.0);
        }
        rho[g] = p;
    }
    orc_set_rho(o, rho);
    free(rho); free(done);
}

void orc_get_rho(const orc *o, double *rho) { orc_density(o, o->f, rho); }

/* velocity, Eq. (11): u[c*Ng + g] */
void orc_get_u(const orc *o, double *u) {
    long Ng = o->Ng;
    for (long g = 0; g < Ng; ++g) {
        double p = 0.0;
        for (int q = 0; q < o->Q; ++q) p += o->f[q * Ng + g];
        for (int c = 0; c < o->dim; ++c) {
            double m = 0.0;
            for (int q = 0; q < o->Q; ++q) m += o->f[q * Ng + g] * o->ev[q][c];
            u[c * Ng + g] = m / p;
        }
    }
}

/* KE_max = max_g 1/2 rho |u|^2 (R14) and mass = sum_g M_A rho */
void orc_diag(const orc *o, double *ke_max, double *mass) {
    long Ng = o->Ng;
    double *rho = malloc(sizeof(double) * Ng), *u = malloc(sizeof(double) * 3 * Ng);
    orc_get_rho(o, rho);
    orc_get_u(o, u);
    double km = 0.0, ms = 0.0;
    for (long g = 0; g < Ng; ++g) {
        double uu = 0.0;
        for (int c = 0; c < o->dim; ++c) uu += u[c * Ng + g] * u[c * Ng + g];
        double ke = 0.5 * rho[g] * uu;
        if (ke > km || ke != ke) km = ke;
        ms += o->MA[g] * rho[g];
    }
    *ke_max = km;
    *mass = ms;
    free(rho); free(u);
}

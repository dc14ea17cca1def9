/*
 * oracle.c -- plain FP64 CPU oracle of the O(a)-improved Wilson-Dirac operator.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links or calls this file;
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant with the HIP path.
 *
 * What it computes (the paper names the operator in the introduction -- "O(a)-improved
 * Wilson fermions", applied as a sparse matrix-vector product -- without writing it out;
 * the form below is the standard Wilson--Sheikholeslami--Wohlert operator, whose free
 * limit is D(p) = m0 + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu):
 *
 *   (D psi)(x) = A(x) psi(x)
 *              - 1/2 sum_mu [ s_mu(x)     U_mu(x)       (1 - gamma_mu) psi(x + mu)
 *                           + s_mu(x - mu) U_mu(x - mu)^+ (1 + gamma_mu) psi(x - mu) ]
 *
 *   A(x) = (4 + m0) 1 + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *   sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],
 *   Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^+) / 8,
 *   Q_{mu nu}(x) = sum of the four counter-clockwise plaquette leaves at x.
 *
 * s_mu(x) = bc_t (-1: antiperiodic) when mu = 0 and x0 = T-1, else +1: the sign sits on
 * fermion hops that cross the time boundary; links themselves are periodic, so the
 * clover term carries no sign.
 *
 * Gamma basis (chiral): gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],[i s_k,0]] in
 * 2x2 blocks, s_k the Pauli matrices; then gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 =
 * diag(1,1,-1,-1).
 *
 * Everything is written with full 4x4 spin matrices and full 3x3 colour matrices, no
 * spin projection, no compression, no even-odd ordering: sites are visited in canonical
 * order ((x0*L1 + x1)*L2 + x2)*L3 + x3 with time slowest.
 *
 * Site loops are OpenMP parallel loops (each iteration writes only its own site, so the
 * result does not depend on the thread count); oracle_set_threads sets the count.
 *
 * Layouts (all complex numbers are interleaved (re, im) doubles):
 *   u    [V][4][3][3]   links U_mu(x) (the full U(3) link: SU(3) part times U(1) phase)
 *   A    [V][12][12]    clover matrix per site, index (spin*3 + colour)
 *   psi  [V][4][3]      spinor field
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static cplx G[4][4][4];       /* gamma_mu[row][col] */
static int gamma_ready = 0;

static void init_gamma(void)
{
    if (gamma_ready) return;
    memset(G, 0, sizeof(G));
    /* Pauli matrices */
    cplx s[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    /* gamma_0: off-diagonal blocks -1 */
    for (int a = 0; a < 2; ++a) {
        G[0][a][2 + a] = -1;
        G[0][2 + a][a] = -1;
    }
    /* gamma_k: upper-right block -i s_k, lower-left block +i s_k */
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                G[k + 1][a][2 + b] = -I * s[k][a][b];
                G[k + 1][2 + a][b] = I * s[k][a][b];
            }
    gamma_ready = 1;
}

/* Export of the basis so that tests can check the Clifford algebra on it. */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int oracle_max_threads(void) { return omp_get_max_threads(); }

void oracle_gamma(double *out /* [4][4][4] complex */)
{
    init_gamma();
    memcpy(out, G, sizeof(G));
}

/* ---------------- geometry ---------------- */

static void coords(const int d[4], long idx, int x[4])
{
    x[3] = (int)(idx % d[3]); idx /= d[3];
    x[2] = (int)(idx % d[2]); idx /= d[2];
    x[1] = (int)(idx % d[1]); idx /= d[1];
    x[0] = (int)idx;
}

static long site_index(const int d[4], const int x[4])
{
    return ((long)(x[0] * (long)d[1] + x[1]) * d[2] + x[2]) * d[3] + x[3];
}

/* neighbour of site idx one step along +mu (dir = +1) or -mu (dir = -1), periodic */
static long step(const int d[4], long idx, int mu, int dir)
{
    int x[4];
    coords(d, idx, x);
    x[mu] = (x[mu] + dir + d[mu]) % d[mu];
    return site_index(d, x);
}

static long volume(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

/* Export of the neighbour map (tests check that every hop round-trips). */
void oracle_neighbours(const int d[4], long *nb /* [V][8]: +0,-0,+1,-1,... */)
{
    long V = volume(d);
    for (long i = 0; i < V; ++i)
        for (int mu = 0; mu < 4; ++mu) {
            nb[i * 8 + 2 * mu] = step(d, i, mu, +1);
            nb[i * 8 + 2 * mu + 1] = step(d, i, mu, -1);
        }
}

/* ---------------- 3x3 colour algebra ---------------- */

static const cplx *link(const cplx *u, long x, int mu) { return u + (x * 4 + mu) * 9; }

static void mat_mul(const cplx *a, const cplx *b, cplx *c)
{
    cplx t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx z = 0;
            for (int k = 0; k < 3; ++k) z += a[i * 3 + k] * b[k * 3 + j];
            t[i * 3 + j] = z;
        }
    memcpy(c, t, sizeof(t));
}

static void mat_dag(const cplx *a, cplx *c)
{
    cplx t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[i * 3 + j] = conj(a[j * 3 + i]);
    memcpy(c, t, sizeof(t));
}

/* ---------------- clover term ---------------- */

/* Q_{mu nu}(x): the four leaves, each a closed counter-clockwise path in the (mu, nu)
 * plane that starts and ends at x. */
static void clover_leaves(const int d[4], const cplx *u, long x, int mu, int nu, cplx *q)
{
    cplx t[9], w[9];
    long xp_mu = step(d, x, mu, +1), xp_nu = step(d, x, nu, +1);
    long xm_mu = step(d, x, mu, -1), xm_nu = step(d, x, nu, -1);
    long xm_mu_p_nu = step(d, xm_mu, nu, +1);
    long xm_mu_m_nu = step(d, xm_mu, nu, -1);
    long xm_nu_p_mu = step(d, xm_nu, mu, +1);
    for (int i = 0; i < 9; ++i) q[i] = 0;

    /* leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
    mat_mul(link(u, x, mu), link(u, xp_mu, nu), t);
    mat_dag(link(u, xp_nu, mu), w); mat_mul(t, w, t);
    mat_dag(link(u, x, nu), w); mat_mul(t, w, t);
    for (int i = 0; i < 9; ++i) q[i] += t[i];

    /* leaf 2: U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu) */
    mat_dag(link(u, xm_mu_p_nu, mu), w); mat_mul(link(u, x, nu), w, t);
    mat_dag(link(u, xm_mu, nu), w); mat_mul(t, w, t);
    mat_mul(t, link(u, xm_mu, mu), t);
    for (int i = 0; i < 9; ++i) q[i] += t[i];

    /* leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu) */
    mat_dag(link(u, xm_mu, mu), t);
    mat_dag(link(u, xm_mu_m_nu, nu), w); mat_mul(t, w, t);
    mat_mul(t, link(u, xm_mu_m_nu, mu), t);
    mat_mul(t, link(u, xm_nu, nu), t);
    for (int i = 0; i < 9; ++i) q[i] += t[i];

    /* leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+ */
    mat_dag(link(u, xm_nu, nu), t);
    mat_mul(t, link(u, xm_nu, mu), t);
    mat_mul(t, link(u, xm_nu_p_mu, nu), t);
    mat_dag(link(u, x, mu), w); mat_mul(t, w, t);
    for (int i = 0; i < 9; ++i) q[i] += t[i];
}

void oracle_clover(const int d[4], const double *u_, double m0, double csw, double *A_)
{
    init_gamma();
    const cplx *u = (const cplx *)u_;
    cplx *A = (cplx *)A_;
    long V = volume(d);

    /* sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] */
    static cplx sig[4][4][4][4];
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx z = 0;
                    for (int k = 0; k < 4; ++k)
                        z += G[mu][a][k] * G[nu][k][b] - G[nu][a][k] * G[mu][k][b];
                    sig[mu][nu][a][b] = 0.5 * I * z;
                }

#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        cplx *Ax = A + x * 144;
        for (int i = 0; i < 144; ++i) Ax[i] = 0;
        for (int i = 0; i < 12; ++i) Ax[i * 12 + i] = 4.0 + m0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) {
                if (mu == nu) continue;
                cplx q[9], F[9];
                clover_leaves(d, u, x, mu, nu, q);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        F[i * 3 + j] = (q[i * 3 + j] - conj(q[j * 3 + i])) / 8.0;
                /* A += c_sw (i/4) sigma_{mu nu} (x) Fhat_{mu nu} */
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        cplx sab = sig[mu][nu][a][b];
                        if (sab == 0) continue;
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j)
                                Ax[(a * 3 + i) * 12 + (b * 3 + j)] +=
                                    csw * 0.25 * I * sab * F[i * 3 + j];
                    }
            }
    }
}

/* ---------------- the Dirac operator ---------------- */

/* out(x) += coef * (U (x) P) v, with U a 3x3 colour matrix (daggered if dag) and P a
 * 4x4 spin matrix acting on v[4][3]. */
static void add_hop(cplx *out, cplx coef, const cplx *U, int dag, const cplx P[4][4],
                    const cplx *v)
{
    for (int s1 = 0; s1 < 4; ++s1)
        for (int c1 = 0; c1 < 3; ++c1) {
            cplx z = 0;
            for (int s2 = 0; s2 < 4; ++s2) {
                if (P[s1][s2] == 0) continue;
                for (int c2 = 0; c2 < 3; ++c2) {
                    cplx uc = dag ? conj(U[c2 * 3 + c1]) : U[c1 * 3 + c2];
                    z += P[s1][s2] * uc * v[s2 * 3 + c2];
                }
            }
            out[s1 * 3 + c1] += coef * z;
        }
}

static double bsign(const int d[4], int bc_t, long x, int mu)
{
    /* sign of the forward hop x -> x + mu */
    if (mu != 0) return 1.0;
    int c[4];
    coords(d, x, c);
    return (c[0] == d[0] - 1) ? (double)bc_t : 1.0;
}

/* block id per coordinate; hops between different blocks are dropped when bs != NULL */
static int same_block(const int d[4], const int *bs, long x, long y)
{
    if (!bs) return 1;
    int a[4], b[4];
    coords(d, x, a);
    coords(d, y, b);
    for (int mu = 0; mu < 4; ++mu)
        if (a[mu] / bs[mu] != b[mu] / bs[mu]) return 0;
    return 1;
}

/* D (adjoint = 0) or the explicit adjoint stencil D^+ (adjoint = 1), optionally
 * restricted to blocks (Dirichlet: hops leaving a block are dropped). */
static void dirac(const int d[4], const int *bs, int bc_t, const cplx *u, const cplx *A,
                  const cplx *psi, cplx *out, int adjoint)
{
    init_gamma();
    long V = volume(d);
    cplx Pm[4][4][4], Pp[4][4][4];     /* 1 - gamma_mu, 1 + gamma_mu */
    for (int mu = 0; mu < 4; ++mu)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx one = (a == b) ? 1.0 : 0.0;
                Pm[mu][a][b] = one - G[mu][a][b];
                Pp[mu][a][b] = one + G[mu][a][b];
            }
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        cplx *o = out + x * 12;
        const cplx *Ax = A + x * 144;
        for (int i = 0; i < 12; ++i) {
            cplx z = 0;
            for (int j = 0; j < 12; ++j)
                z += (adjoint ? conj(Ax[j * 12 + i]) : Ax[i * 12 + j]) * psi[x * 12 + j];
            o[i] = z;
        }
        for (int mu = 0; mu < 4; ++mu) {
            long xf = step(d, x, mu, +1), xb = step(d, x, mu, -1);
            const cplx(*Pf)[4] = adjoint ? Pp[mu] : Pm[mu];
            const cplx(*Pb)[4] = adjoint ? Pm[mu] : Pp[mu];
            if (same_block(d, bs, x, xf))
                add_hop(o, -0.5 * bsign(d, bc_t, x, mu), link(u, x, mu), 0, Pf,
                        psi + xf * 12);
            if (same_block(d, bs, x, xb))
                add_hop(o, -0.5 * bsign(d, bc_t, xb, mu), link(u, xb, mu), 1, Pb,
                        psi + xb * 12);
        }
    }
}

void oracle_dw(const int d[4], int bc_t, const double *u, const double *A,
               const double *psi, double *out)
{
    dirac(d, NULL, bc_t, (const cplx *)u, (const cplx *)A, (const cplx *)psi, (cplx *)out, 0);
}

void oracle_dw_dag(const int d[4], int bc_t, const double *u, const double *A,
                   const double *psi, double *out)
{
    dirac(d, NULL, bc_t, (const cplx *)u, (const cplx *)A, (const cplx *)psi, (cplx *)out, 1);
}

/* Direct sum over all blocks of the block-restricted operators D_b (every block at once;
 * a hop whose two ends lie in different blocks is dropped). */
void oracle_dw_blocks(const int d[4], const int bs[4], int bc_t, const double *u,
                      const double *A, const double *psi, double *out)
{
    dirac(d, bs, bc_t, (const cplx *)u, (const cplx *)A, (const cplx *)psi, (cplx *)out, 0);
}

/* Gauge links as full U(3) matrices: U = exp(i theta) V. */
void oracle_u3_links(long V, const double *su3_, const double *theta, double *u_)
{
    const cplx *su3 = (const cplx *)su3_;
    cplx *u = (cplx *)u_;
#pragma omp parallel for schedule(static)
    for (long l = 0; l < V * 4; ++l) {
        cplx ph = cexp(I * theta[l]);
        for (int i = 0; i < 9; ++i) u[l * 9 + i] = ph * su3[l * 9 + i];
    }
}

/* (D psi)(x) at a list of sites only, with the clover term built at those sites: lets a
 * test sample outputs of a lattice too large for a full oracle sweep. */
void oracle_dw_at(const int d[4], int bc_t, const double *u_, double m0, double csw,
                  const double *psi_, const long *sites, long n, double *out_ /* [n][12] */)
{
    init_gamma();
    const cplx *u = (const cplx *)u_;
    const cplx *psi = (const cplx *)psi_;
    cplx *out = (cplx *)out_;
    /* clover of one site: reuse oracle_clover on a one-site view is not possible (it
     * needs neighbours), so rebuild A(x) here with the same definition */
    static cplx sig[4][4][4][4];
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx z = 0;
                    for (int k = 0; k < 4; ++k)
                        z += G[mu][a][k] * G[nu][k][b] - G[nu][a][k] * G[mu][k][b];
                    sig[mu][nu][a][b] = 0.5 * I * z;
                }
    cplx Pm[4][4][4], Pp[4][4][4];
    for (int mu = 0; mu < 4; ++mu)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx one = (a == b) ? 1.0 : 0.0;
                Pm[mu][a][b] = one - G[mu][a][b];
                Pp[mu][a][b] = one + G[mu][a][b];
            }
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        long x = sites[k];
        cplx Ax[144];
        for (int i = 0; i < 144; ++i) Ax[i] = 0;
        for (int i = 0; i < 12; ++i) Ax[i * 12 + i] = 4.0 + m0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) {
                if (mu == nu) continue;
                cplx q[9], F[9];
                clover_leaves(d, u, x, mu, nu, q);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        F[i * 3 + j] = (q[i * 3 + j] - conj(q[j * 3 + i])) / 8.0;
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        cplx sab = sig[mu][nu][a][b];
                        if (sab == 0) continue;
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j)
                                Ax[(a * 3 + i) * 12 + (b * 3 + j)] +=
                                    csw * 0.25 * I * sab * F[i * 3 + j];
                    }
            }
        cplx *o = out + k * 12;
        for (int i = 0; i < 12; ++i) {
            cplx z = 0;
            for (int j = 0; j < 12; ++j) z += Ax[i * 12 + j] * psi[x * 12 + j];
            o[i] = z;
        }
        for (int mu = 0; mu < 4; ++mu) {
            long xf = step(d, x, mu, +1), xb = step(d, x, mu, -1);
            add_hop(o, -0.5 * bsign(d, bc_t, x, mu), link(u, x, mu), 0, Pm[mu], psi + xf * 12);
            add_hop(o, -0.5 * bsign(d, bc_t, xb, mu), link(u, xb, mu), 1, Pp[mu], psi + xb * 12);
        }
    }
}

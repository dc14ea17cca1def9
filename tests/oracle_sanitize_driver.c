/* Runs every C routine of the oracle once on a small lattice, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py): an
 * out-of-bounds access, a use of freed memory, a leak or an undefined operation ends the
 * program with a report. It also checks two identities of the results, so that the run
 * is not vacuous: D^+ is the adjoint of D (<phi, D psi> = <D^+ phi, psi>), and the
 * site-sampled D equals the full D at every site. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_set_threads(int n);
void oracle_gamma(double *out);
void oracle_neighbours(const int d[4], long *nb);
void oracle_clover(const int d[4], const double *u, double m0, double csw, double *A);
void oracle_dw(const int d[4], int bc_t, const double *u, const double *A, const double *psi,
               double *out);
void oracle_dw_dag(const int d[4], int bc_t, const double *u, const double *A,
                   const double *psi, double *out);
void oracle_dw_blocks(const int d[4], const int bs[4], int bc_t, const double *u,
                      const double *A, const double *psi, double *out);
void oracle_u3_links(long V, const double *su3, const double *theta, double *u);
void oracle_dw_at(const int d[4], int bc_t, const double *u, double m0, double csw,
                  const double *psi, const long *sites, long n, double *out);

/* xorshift64*, uniform in [-1, 1) */
static unsigned long long rng_state = 0x9E3779B97F4A7C15ULL;
static double uniform(void)
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    const unsigned long long r = rng_state * 2685821657736338717ULL;
    return (double)(r >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static double *alloc_fill(long n)
{
    double *p = malloc(sizeof(double) * n);
    if (!p) exit(2);
    for (long i = 0; i < n; ++i) p[i] = uniform();
    return p;
}

static double complex dot(const double *a, const double *b, long n /* complex entries */)
{
    double complex s = 0;
    for (long i = 0; i < n; ++i)
        s += conj(a[2 * i] + I * a[2 * i + 1]) * (b[2 * i] + I * b[2 * i + 1]);
    return s;
}

int main(void)
{
    const int d[4] = {6, 4, 4, 6};
    const int bs[4] = {2, 2, 2, 2};
    const long V = (long)d[0] * d[1] * d[2] * d[3];
    const long nsp = V * 12; /* complex entries of a spinor field */
    oracle_set_threads(2);

    double g[4 * 4 * 4 * 2];
    oracle_gamma(g);
    long *nb = malloc(sizeof(long) * V * 8);
    if (!nb) return 2;
    oracle_neighbours(d, nb);
    for (long i = 0; i < V * 8; ++i)
        if (nb[i] < 0 || nb[i] >= V) return 3;

    double *su3 = alloc_fill(V * 4 * 9 * 2), *theta = alloc_fill(V * 4);
    double *u = malloc(sizeof(double) * V * 4 * 9 * 2);
    double *A = malloc(sizeof(double) * V * 144 * 2);
    if (!u || !A) return 2;
    oracle_u3_links(V, su3, theta, u);
    oracle_clover(d, u, 0.1, 1.7, A);

    double *psi = alloc_fill(nsp * 2), *phi = alloc_fill(nsp * 2);
    double *Dpsi = malloc(sizeof(double) * nsp * 2), *Dphi = malloc(sizeof(double) * nsp * 2);
    double *Bpsi = malloc(sizeof(double) * nsp * 2), *at = malloc(sizeof(double) * nsp * 2);
    long *sites = malloc(sizeof(long) * V);
    if (!Dpsi || !Dphi || !Bpsi || !at || !sites) return 2;
    oracle_dw(d, -1, u, A, psi, Dpsi);
    oracle_dw_dag(d, -1, u, A, phi, Dphi);
    oracle_dw_blocks(d, bs, -1, u, A, psi, Bpsi);
    for (long x = 0; x < V; ++x) sites[x] = x;
    oracle_dw_at(d, -1, u, 0.1, 1.7, psi, sites, V, at);

    const double complex lhs = dot(phi, Dpsi, nsp), rhs = dot(Dphi, psi, nsp);
    const double adj = cabs(lhs - rhs) / cabs(lhs);
    double sampled = 0.0, scale = 0.0;
    for (long i = 0; i < nsp * 2; ++i) {
        sampled = fmax(sampled, fabs(at[i] - Dpsi[i]));
        scale = fmax(scale, fabs(Dpsi[i]));
    }
    free(nb); free(su3); free(theta); free(u); free(A); free(psi); free(phi);
    free(Dpsi); free(Dphi); free(Bpsi); free(at); free(sites);
    if (!(adj < 1e-12) || !(sampled <= 1e-13 * scale)) {
        printf("identity failed: adjoint %.3e, sampled %.3e\n", adj, sampled / scale);
        return 4;
    }
    printf("ok adjoint %.3e sampled %.3e\n", adj, sampled / scale);
    return 0;
}

/*
 * Plain C state-vector loops for the CPU oracle (test infrastructure only).
 *
 * Same mathematics as oracle/statevec.py, written as one OpenMP loop over
 * basis states per Pauli string so that 20-28 qubit references finish on a
 * host.  Nothing here is fused, blocked or reordered beyond one pass per
 * string (apply) or per flip-mask group (energy: the strings of a group share
 * the partner amplitude psi[b ^ x], Sec. 3.1 Eq. (17) summed group by group).
 *
 * Conventions: psi is complex128 stored as interleaved (re, im) doubles,
 * amplitude index b has qubit q at bit q (Sec. 2.1.1, Eq. (3)).
 * P(x, z)|b> = i^popcount(x & z) (-1)^popcount(b & z) |b ^ x>.
 * exp(-i theta P) = cos(theta) - i sin(theta) P.
 * Sums use Neumaier compensation per thread and a fixed-order combine, so a
 * run with a given thread count is reproducible.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

typedef struct { double s, c; } nsum;

static inline void nadd(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static inline int parity64(uint64_t v) { return __builtin_popcountll(v) & 1; }

/* omega(b) = i^k: returns k in 0..3 */
static inline int omega_k(uint64_t x, uint64_t z, uint64_t b)
{
    return (__builtin_popcountll(x & z) + 2 * parity64(b & z)) & 3;
}

/* multiply (re, im) by i^k */
static inline void mul_ik(int k, double re, double im, double *ore, double *oim)
{
    switch (k) {
    case 0: *ore = re; *oim = im; break;
    case 1: *ore = -im; *oim = re; break;
    case 2: *ore = -re; *oim = -im; break;
    default: *ore = im; *oim = -re; break;
    }
}

int orc_threads(void) { return omp_get_max_threads(); }

void orc_set_threads(int n) { omp_set_num_threads(n); }

void orc_prepare(double *psi, int n, uint64_t occ)
{
    int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < 2 * dim; b++)
        psi[b] = 0.0;
    psi[2 * occ] = 1.0;
}

/* psi <- exp(-i theta P(x,z)) psi, in place */
void orc_apply_exp(double *psi, int n, uint64_t x, uint64_t z, double theta)
{
    int64_t dim = (int64_t)1 << n;
    double cs = cos(theta), sn = sin(theta);
    if (x == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < dim; b++) {
            int k = omega_k(x, z, (uint64_t)b);
            double wr, wi; /* -i sin * omega */
            mul_ik((k + 3) & 3, sn, 0.0, &wr, &wi);
            double fr = cs + wr, fi = wi;
            double re = psi[2 * b], im = psi[2 * b + 1];
            psi[2 * b] = fr * re - fi * im;
            psi[2 * b + 1] = fr * im + fi * re;
        }
        return;
    }
    uint64_t hb = (uint64_t)1 << (63 - __builtin_clzll(x));
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < dim; b++) {
        uint64_t y = (uint64_t)b;
        if (y & hb)
            continue;
        uint64_t y2 = y ^ x;
        double ar = psi[2 * y], ai = psi[2 * y + 1];
        double br = psi[2 * y2], bi = psi[2 * y2 + 1];
        /* (P psi)[y] = omega(y2) psi[y2]; (P psi)[y2] = omega(y) psi[y] */
        double pr, pi, qr, qi;
        mul_ik(omega_k(x, z, y2), br, bi, &pr, &pi);
        mul_ik(omega_k(x, z, y), ar, ai, &qr, &qi);
        /* new = cs * old - i sn * P-part ; -i*(r + i m) = m - i r */
        psi[2 * y] = cs * ar + sn * pi;
        psi[2 * y + 1] = cs * ai - sn * pr;
        psi[2 * y2] = cs * br + sn * qi;
        psi[2 * y2 + 1] = cs * bi - sn * qr;
    }
}

void orc_apply_product(double *psi, int n, const uint64_t *xs, const uint64_t *zs,
                       const double *th, int64_t K, int inverse)
{
    if (!inverse) {
        for (int64_t k = 0; k < K; k++)
            orc_apply_exp(psi, n, xs[k], zs[k], th[k]);
    } else {
        for (int64_t k = K - 1; k >= 0; k--)
            orc_apply_exp(psi, n, xs[k], zs[k], -th[k]);
    }
}

/* sum over groups g of sum_b Re( conj(psi[b^x_g]) * (sum_{k in g} c_k omega_k(b)) * psi[b] ) */
double orc_energy(const double *psi, int n, const uint64_t *xs, const uint64_t *zs,
                  const double *cs, const int64_t *goff, int64_t G)
{
    int64_t dim = (int64_t)1 << n;
    int nt = omp_get_max_threads();
    nsum *part = (nsum *)calloc((size_t)nt, sizeof(nsum));
#pragma omp parallel
    {
        nsum acc = {0.0, 0.0};
        for (int64_t g = 0; g < G; g++) {
            uint64_t x = xs[goff[g]];
#pragma omp for schedule(static)
            for (int64_t b = 0; b < dim; b++) {
                uint64_t y = (uint64_t)b;
                double dr = 0.0, di = 0.0;
                for (int64_t k = goff[g]; k < goff[g + 1]; k++) {
                    double wr, wi;
                    mul_ik(omega_k(x, zs[k], y), cs[k], 0.0, &wr, &wi);
                    dr += wr;
                    di += wi;
                }
                uint64_t y2 = y ^ x;
                double ar = psi[2 * y], ai = psi[2 * y + 1];
                double br = psi[2 * y2], bi = psi[2 * y2 + 1];
                /* t = D * a ; contrib = Re(conj(b) * t) */
                double tr = dr * ar - di * ai, ti = dr * ai + di * ar;
                nadd(&acc, br * tr + bi * ti);
            }
        }
        part[omp_get_thread_num()] = acc;
    }
    nsum tot = {0.0, 0.0};
    for (int t = 0; t < nt; t++) {
        nadd(&tot, part[t].s);
        nadd(&tot, part[t].c);
    }
    free(part);
    return tot.s + tot.c;
}

/* out = sum_k c_k P_k psi  (out is overwritten) */
void orc_sigma(const double *psi, double *out, int n, const uint64_t *xs, const uint64_t *zs,
               const double *cs, int64_t K)
{
    int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < 2 * dim; b++)
        out[b] = 0.0;
    for (int64_t k = 0; k < K; k++) {
        uint64_t x = xs[k], z = zs[k];
        double c = cs[k];
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < dim; b++) {
            /* out[b] += c * omega(b ^ x) * psi[b ^ x] */
            uint64_t y2 = (uint64_t)b ^ x;
            double pr, pi;
            mul_ik(omega_k(x, z, y2), psi[2 * y2], psi[2 * y2 + 1], &pr, &pi);
            out[2 * b] += c * pr;
            out[2 * b + 1] += c * pi;
        }
    }
}

/* <a|b> real and imaginary parts, compensated */
void orc_vdot(const double *a, const double *b, int n, double *re, double *im)
{
    int64_t dim = (int64_t)1 << n;
    int nt = omp_get_max_threads();
    nsum *pr = (nsum *)calloc((size_t)nt, sizeof(nsum));
    nsum *pi = (nsum *)calloc((size_t)nt, sizeof(nsum));
#pragma omp parallel
    {
        nsum r = {0, 0}, m = {0, 0};
#pragma omp for schedule(static)
        for (int64_t y = 0; y < dim; y++) {
            double ar = a[2 * y], ai = a[2 * y + 1], br = b[2 * y], bi = b[2 * y + 1];
            nadd(&r, ar * br + ai * bi);
            nadd(&m, ar * bi - ai * br);
        }
        pr[omp_get_thread_num()] = r;
        pi[omp_get_thread_num()] = m;
    }
    nsum R = {0, 0}, M = {0, 0};
    for (int t = 0; t < nt; t++) {
        nadd(&R, pr[t].s); nadd(&R, pr[t].c);
        nadd(&M, pi[t].s); nadd(&M, pi[t].c);
    }
    free(pr);
    free(pi);
    *re = R.s + R.c;
    *im = M.s + M.c;
}

/* Im <lam| P(x,z) |phi> */
static double im_expval(const double *lam, const double *phi, int n, uint64_t x, uint64_t z)
{
    int64_t dim = (int64_t)1 << n;
    int nt = omp_get_max_threads();
    nsum *part = (nsum *)calloc((size_t)nt, sizeof(nsum));
#pragma omp parallel
    {
        nsum acc = {0, 0};
#pragma omp for schedule(static)
        for (int64_t b = 0; b < dim; b++) {
            /* (P phi)[y2] = omega(b) phi[b], y2 = b ^ x; term conj(lam[y2]) * that */
            uint64_t y2 = (uint64_t)b ^ x;
            double pr, pi;
            mul_ik(omega_k(x, z, (uint64_t)b), phi[2 * b], phi[2 * b + 1], &pr, &pi);
            double lr = lam[2 * y2], li = lam[2 * y2 + 1];
            nadd(&acc, lr * pi - li * pr);
        }
        part[omp_get_thread_num()] = acc;
    }
    nsum tot = {0, 0};
    for (int t = 0; t < nt; t++) {
        nadd(&tot, part[t].s);
        nadd(&tot, part[t].c);
    }
    free(part);
    return tot.s + tot.c;
}

/*
 * Energy and dE/dtheta_k for psi = U_{K-1}...U_0 |occ>, U_k = exp(-i theta_k P_k):
 * lambda = H psi, then for k = K-1..0: g_k = 2 Im <lambda|P_k|phi>, and both
 * phi and lambda are multiplied by U_k^dagger.  work holds two states.
 */
void orc_energy_grad(int n, uint64_t occ, const uint64_t *ax, const uint64_t *az, const double *th,
                     int64_t K, const uint64_t *hx, const uint64_t *hz, const double *hc, int64_t KH,
                     double *work, double *E, double *grad)
{
    int64_t dim = (int64_t)1 << n;
    double *phi = work;
    double *lam = work + 2 * dim;
    orc_prepare(phi, n, occ);
    orc_apply_product(phi, n, ax, az, th, K, 0);
    orc_sigma(phi, lam, n, hx, hz, hc, KH);
    double re, im;
    orc_vdot(phi, lam, n, &re, &im);
    *E = re;
    for (int64_t k = K - 1; k >= 0; k--) {
        grad[k] = 2.0 * im_expval(lam, phi, n, ax[k], az[k]);
        orc_apply_exp(phi, n, ax[k], az[k], -th[k]);
        orc_apply_exp(lam, n, ax[k], az[k], -th[k]);
    }
}

/*
 * ADAPT pool gradients (Sec. 3.2): for each pool member nu with strings
 * off[nu] .. off[nu+1], g[nu] = -2 sum_k c_k Im <lam|P_k|psi>, which is
 * 2 Re <lam|kappa_nu psi> for JW(kappa_nu) = i sum_k c_k P_k and lam = H psi.
 */
void orc_pool_grad(const double *psi, const double *lam, int n, const uint64_t *xs, const uint64_t *zs,
                   const double *cs, const int64_t *off, int64_t npool, double *g)
{
    for (int64_t nu = 0; nu < npool; nu++) {
        nsum acc = {0.0, 0.0};
        for (int64_t k = off[nu]; k < off[nu + 1]; k++)
            nadd(&acc, -2.0 * cs[k] * im_expval(lam, psi, n, xs[k], zs[k]));
        g[nu] = acc.s + acc.c;
    }
}

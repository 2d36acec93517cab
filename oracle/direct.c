/*
 * FP64 direct-summation oracle for the regularised vortex-particle sums.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the bench do.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (Yokota, Barba, Narumi, Yasuoka, "Petascale turbulence
 * simulation using a highly parallel fast multipole method on GPUs",
 * Sec. 2.1, Eqs. (1)-(3)):
 *
 *   For a target i and every source j (and every periodic shift n in the given
 *   list), with r = x_i - x_j - n, rho = |r|, sigma = sigma_j (the source core,
 *   Eq. (2)), s = rho / (sqrt(2) sigma):
 *
 *     g(s)   = erf(s) - (2/sqrt(pi)) s exp(-s^2)          cutoff, Eq. (2)
 *     q      = g / (4 pi rho^3)
 *     dq/drho / rho = (sqrt(2/pi) (rho/sigma)^3 exp(-s^2) - 3 g) / (4 pi rho^5)
 *
 *     u_i    += q * (alpha_j x r)                          Biot-Savart, Eq. (1)
 *     J_i,kl += q eps_{l m k} alpha_j,m + (q'/rho) r_k (alpha_j x r)_l
 *
 *   J_kl = d u_l / d x_k is the velocity gradient at the target; the
 *   stretching term of Eq. (3) is a contraction of J with alpha_i, done by the
 *   Python wrapper.
 *
 * Sign: u = curl psi with -lap psi = omega, i.e. the physical Biot-Savart law
 * u(x) = (1/4pi) sum alpha_j x (x - x_j) / |x - x_j|^3 for far pairs.
 *
 * r -> 0 (self pair, coincident particles): q and q'/rho are replaced by
 * their Taylor series in s (the exact expansion of the definitions above),
 * used for rho/sigma < 0.5 so that no cancellation or 0/0 occurs; at rho = 0
 * the series gives the finite limit.
 */
#include <math.h>
#include <stdint.h>

#define PI_D 3.14159265358979323846

/* q and q'/rho for one pair.  Series branch: with c = 1/(sqrt(2) sigma),
 *   q      = c^3/(4 pi) (4/sqrt(pi)) sum_{n>=0} (-1)^n s^{2n} / (n! (2n+3))
 *   q'/rho = c^5/(4 pi) (4/sqrt(pi)) sum_{n>=1} (-1)^n 2 s^{2n-2} / ((n-1)! (2n+3))
 * which follow from term-wise expansion of erf and exp in g(s). */
static void pair_factors(double rho2, double sigma, double *q, double *qpr)
{
    const double rho = sqrt(rho2);
    const double c = 1.0 / (sqrt(2.0) * sigma);
    const double s = rho * c;
    const double four_over_sqrtpi = 4.0 / sqrt(PI_D);
    if (rho < 0.5 * sigma) {
        const double s2 = s * s;
        double f = 0.0, h = 0.0;
        double pw = 1.0, fact = 1.0;        /* s^{2n} and n!           */
        double pwm = 1.0, factm = 1.0;      /* s^{2n-2} and (n-1)!     */
        for (int n = 0; n <= 24; ++n) {
            const double sg = (n & 1) ? -1.0 : 1.0;
            f += sg * pw / (fact * (2.0 * n + 3.0));
            if (n >= 1) {
                h += sg * 2.0 * pwm / (factm * (2.0 * n + 3.0));
                pwm = pw;
                factm = fact;
            }
            pw *= s2;
            fact *= (n + 1);
        }
        const double c3 = c * c * c;
        *q = c3 / (4.0 * PI_D) * four_over_sqrtpi * f;
        *qpr = c3 * c * c / (4.0 * PI_D) * four_over_sqrtpi * h;
    } else {
        const double e = exp(-s * s);
        const double g = erf(s) - (2.0 / sqrt(PI_D)) * s * e;
        const double rho3 = rho2 * rho;
        const double ros = rho / sigma;
        *q = g / (4.0 * PI_D * rho3);
        *qpr = (sqrt(2.0 / PI_D) * ros * ros * ros * e - 3.0 * g) / (4.0 * PI_D * rho3 * rho2);
    }
}

/* Exported for the pins that check the cutoff factors alone. */
void oracle_pair_factors(int64_t n, const double *rho, const double *sigma, double *q, double *qpr)
{
    for (int64_t i = 0; i < n; ++i)
        pair_factors(rho[i] * rho[i], sigma[i], &q[i], &qpr[i]);
}

/*
 * u[3*i+l] and J[9*i + 3*k + l] for targets i in [0, nt), summed over all
 * sources j in [0, ns) and all shifts (nshift triples; pass nshift = 0 and
 * shifts = NULL for free space).  Parallel over targets; each target's sum
 * runs sources in index order, shifts outermost.
 */
void oracle_direct(int64_t nt, const double *tx, const double *ty, const double *tz,
                   int64_t ns, const double *sx, const double *sy, const double *sz,
                   const double *sax, const double *say, const double *saz, const double *ssig,
                   int64_t nshift, const double *shifts, double *u, double *J)
{
    const int64_t nsh = nshift > 0 ? nshift : 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double ui[3] = {0, 0, 0};
        double Ji[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t t = 0; t < nsh; ++t) {
            const double shx = nshift > 0 ? shifts[3 * t + 0] : 0.0;
            const double shy = nshift > 0 ? shifts[3 * t + 1] : 0.0;
            const double shz = nshift > 0 ? shifts[3 * t + 2] : 0.0;
            for (int64_t j = 0; j < ns; ++j) {
                const double r[3] = {tx[i] - sx[j] - shx, ty[i] - sy[j] - shy, tz[i] - sz[j] - shz};
                const double a[3] = {sax[j], say[j], saz[j]};
                const double rho2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                double q, qpr;
                pair_factors(rho2, ssig[j], &q, &qpr);
                /* alpha_j x r */
                const double axr[3] = {a[1] * r[2] - a[2] * r[1],
                                       a[2] * r[0] - a[0] * r[2],
                                       a[0] * r[1] - a[1] * r[0]};
                for (int l = 0; l < 3; ++l)
                    ui[l] += q * axr[l];
                /* q eps_{l m k} a_m : the matrix with (k,l) entry sum_m eps_{lmk} a_m */
                /* eps_{lmk} a_m for (k,l):  (k=0,l=1)->eps_{1,2,0} a_2 = +a2 ; etc. */
                for (int k = 0; k < 3; ++k) {
                    for (int l = 0; l < 3; ++l) {
                        double e = 0.0;
                        for (int m = 0; m < 3; ++m) {
                            /* Levi-Civita eps_{l m k} */
                            int p = (l == m || m == k || l == k) ? 0
                                    : (((l + 1) % 3 == m) ? 1 : -1);
                            e += p * a[m];
                        }
                        Ji[3 * k + l] += q * e + qpr * r[k] * axr[l];
                    }
                }
            }
        }
        for (int l = 0; l < 3; ++l)
            u[3 * i + l] = ui[l];
        for (int k = 0; k < 9; ++k)
            J[9 * i + k] = Ji[k];
    }
}

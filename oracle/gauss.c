/*
 * FP64 direct sum of the Gaussian blob kernel, for the radial-basis-function
 * reinitialisation of the particle strengths.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it shares no code, header or constant with the HIP library.
 *
 * The blobs of Eq. (2) carry the normalised Gaussian vorticity distribution
 * zeta_sigma whose enclosed mass is the cutoff g (Sec. 2.1):
 *
 *     zeta_s(r) = (2 pi s^2)^(-3/2) exp(-r^2 / (2 s^2)),
 *
 * and the vorticity represented by particles of strengths gamma_j at a point
 * x is sum_j gamma_j zeta_{sigma_j}(x - x_j).  Reinitialising the particles
 * (Sec. 2.1, last paragraph; Sec. 2.2) asks for strengths that reproduce a
 * given vorticity at the particle positions, a linear system whose matrix is
 * this sum.
 */
#include <math.h>
#include <stdint.h>

#define PI_D 3.14159265358979323846

/*
 * out[3*i + c] = sum over shifts n and sources j of
 *                gamma_c[j] zeta_{sig[j]}(t_i - s_j - shift_n)
 * for targets i in [0, nt); nshift = 0 (shifts = NULL) means free space.
 * Parallel over targets; each target sums shifts outermost, sources in order.
 */
void oracle_gauss_sum(int64_t nt, const double *tx, const double *ty, const double *tz,
                      int64_t ns, const double *sx, const double *sy, const double *sz,
                      const double *gx, const double *gy, const double *gz, const double *sig,
                      int64_t nshift, const double *shifts, double *out)
{
    const int64_t nsh = nshift > 0 ? nshift : 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t t = 0; t < nsh; ++t) {
            const double shx = nshift > 0 ? shifts[3 * t + 0] : 0.0;
            const double shy = nshift > 0 ? shifts[3 * t + 1] : 0.0;
            const double shz = nshift > 0 ? shifts[3 * t + 2] : 0.0;
            for (int64_t j = 0; j < ns; ++j) {
                const double dx = tx[i] - sx[j] - shx, dy = ty[i] - sy[j] - shy, dz = tz[i] - sz[j] - shz;
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double s2 = sig[j] * sig[j];
                const double z = pow(2.0 * PI_D * s2, -1.5) * exp(-0.5 * r2 / s2);
                acc[0] += gx[j] * z;
                acc[1] += gy[j] * z;
                acc[2] += gz[j] * z;
            }
        }
        out[3 * i + 0] = acc[0];
        out[3 * i + 1] = acc[1];
        out[3 * i + 2] = acc[2];
    }
}

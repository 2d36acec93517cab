// Periodic lattice operator (Sec. 3.5): the contribution of the far periodic
// images to the root local expansion, as one real-linear map of the root
// multipole, built once in float64 on the host.
//
// The traversal treats the images |n|_inf <= 4 explicitly (9 periods per
// axis).  Images further out are grouped into cubic supercells: S_0 is the
// box, S_j = 3 x 3 x 3 copies of S_{j-1} (multipole by M2M of the 27 copies).
// Level j >= 2 adds the shell S_{j+1} \ S_j, made of the copies of S_{j-2}
// at offsets o (in units of S_{j-2}) with o in {-13..13}^3 \ {-4..4}^3, via
// M2L into the root.  With K levels (images = K) the sum covers
// |n|_inf <= (3^K - 1) / 2 in cube order.  All operators are written for the
// size-normalised expansions, in which both the supercell M2M and the ring M2L
// are the same for every level up to a diagonal rescaling.
#include <complex>
#include <vector>

#include "ctx.h"

namespace vfmm {

using cd = std::complex<double>;

static inline cd getcd(const std::vector<cd> &a, int n, int m) {
    if (m >= 0) return a[CIDX(n, m)];
    const cd v = std::conj(a[CIDX(n, -m)]);
    return (m & 1) ? -v : v;
}

template <int P>
static void lattice_op_p(int K, std::vector<double> &op) {
    constexpr int NCP = NC(P);
    constexpr int Q = 2 * P;
    constexpr int NCQ = NC(Q);
    const int D = 2 * NCP;
    op.assign((size_t)D * D, 0.0);
    if (K < 3) return;
    // ring sum of irregular harmonics
    std::vector<cd> S(NCQ, cd(0, 0)), I(NCQ);
    for (int ox = -13; ox <= 13; ++ox)
        for (int oy = -13; oy <= 13; ++oy)
            for (int oz = -13; oz <= 13; ++oz) {
                if (std::abs(ox) <= 4 && std::abs(oy) <= 4 && std::abs(oz) <= 4) continue;
                irregular_harmonics<Q, double, cd>((double)ox, (double)oy, (double)oz, I.data());
                for (int t = 0; t < NCQ; ++t) S[t] += I[t];
            }
    // 27-copy supercell translation: sum_d conj(R(d/3))
    std::vector<cd> SR(NCP, cd(0, 0)), R(NCP);
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                regular_harmonics<P, double, cd>(dx / 3.0, dy / 3.0, dz / 3.0, R.data());
                for (int t = 0; t < NCP; ++t) SR[t] += std::conj(R[t]);
            }
    auto apply_A = [&](const std::vector<cd> &M) {
        std::vector<cd> out(NCP, cd(0, 0));
        for (int n = 0; n <= P; ++n)
            for (int m = 0; m <= n; ++m) {
                cd acc(0, 0);
                for (int k = n; k >= 0; --k) {
                    const int nm = n - k;
                    const double sc = std::pow(3.0, -nm);
                    for (int l = -k; l <= k; ++l) {
                        const int mm = m - l;
                        if (mm < -nm || mm > nm) continue;
                        acc += getcd(SR, k, l) * getcd(M, nm, mm) * sc;
                    }
                }
                out[CIDX(n, m)] = acc;
            }
        return out;
    };
    auto apply_T = [&](const std::vector<cd> &M) {
        std::vector<cd> out(NCP, cd(0, 0));
        for (int k = 0; k <= P; ++k)
            for (int l = 0; l <= k; ++l) {
                cd acc(0, 0);
                for (int n = P; n >= 0; --n)
                    for (int m = -n; m <= n; ++m) acc += getcd(M, n, m) * getcd(S, n + k, m - l);
                out[CIDX(k, l)] = ((k + l) & 1) ? -acc : acc;
            }
        return out;
    };
    for (int b = 0; b < D; ++b) {
        const int coef = b / 2, part = b % 2;
        int nn = 0;
        while ((nn + 1) * (nn + 2) / 2 <= coef) ++nn;
        const int mm = coef - nn * (nn + 1) / 2;
        if (part == 1 && mm == 0) continue;  // Im of an m = 0 coefficient of a real field is zero
        std::vector<cd> M(NCP, cd(0, 0)), L(NCP, cd(0, 0));
        M[coef] = part ? cd(0, 1) : cd(1, 0);
        for (int j = 2; j <= K - 1; ++j) {
            const std::vector<cd> Lj = apply_T(M);
            for (int k = 0; k <= P; ++k) {
                const double sc = std::pow(3.0, -(double)(j - 2) * (k + 1));
                for (int l = 0; l <= k; ++l) L[CIDX(k, l)] += sc * Lj[CIDX(k, l)];
            }
            if (j < K - 1) M = apply_A(M);
        }
        for (int r = 0; r < D; ++r) op[(size_t)r * D + b] = (r & 1) ? L[r / 2].imag() : L[r / 2].real();
    }
}

void lattice_operator_host(int p, int K, std::vector<double> &op) {
    switch (p) {
        case 4: lattice_op_p<4>(K, op); break;
        case 6: lattice_op_p<6>(K, op); break;
        case 8: lattice_op_p<8>(K, op); break;
        case 10: lattice_op_p<10>(K, op); break;
        case 12: lattice_op_p<12>(K, op); break;
        default: throw Error{VFMM_EINVAL, "unsupported expansion degree p"};
    }
}

}  // namespace vfmm

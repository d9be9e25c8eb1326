/*
 * FP64 CPU oracle for TNEP tensor evaluation (arXiv:2312.05233).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Plain, slow, obviously-correct definitions, in double precision:
 *   - site-energy decomposition U = sum_i U_i(q_i)              (Sec. 2.1, Eq. site-energy)
 *   - virial  W = -sum_i sum_{j!=i} r_ij (x) dU_i/dr_ij         (Sec. 2.1, Eq. virial)
 *   - dipole  mu = -sum_i sum_{j!=i} r_ij^2 dU_i/dr_ij          (Sec. 2.2, Eq. mu)
 *   - polarizability alpha = sum_i U_i I + W                    (Sec. 2.3, Eq. polarizability-model)
 *   - potential-energy surface (Sec. 2.1): energy U, virial W and forces
 *     F_k = -dU/dr_k = sum_j dU_k/dr_kj - sum_i dU_i/dr_ik
 * with r_ij = r_j - r_i (Sec. 2.1, text after Eq. virial).
 *
 * The descriptor q_i is only cited by the paper (NEP, Sec. 2.1); this file
 * follows the reading recorded with the project design:
 *   f_c(r)   = (1 + cos(pi r / r_c)) / 2  for r < r_c, else 0
 *   x(r)     = 2 (r / r_c - 1)^2 - 1
 *   f_k(r)   = (T_k(x) + 1) / 2 * f_c(r),  k = 0..K  (Chebyshev, 1st kind)
 *   g_n(r)   = sum_k c^{t_i t_j}_{nk} f_k(r)
 *   q^R_n    = sum_{j: r<rc_R} g^R_n(r_ij)
 *   A_nlm    = sum_{j: r<rc_A} g^A_n(r_ij) Y_lm(r_ij / r_ij), real orthonormal Y_lm
 *   q_nl     = sum_m A_nlm^2                     (l = 1..l_max)
 *   q4_n     = sum_{m1+m2+m3=0} (2 2 2; m1 m2 m3) At_{n2m1} At_{n2m2} At_{n2m3}
 *              with At the complex-basis (Condon-Shortley) sums
 *   q5_n     = (sum_m A_n1m^2)^2  (optional five-body term: the only degree-4
 *              rotation invariant of the l = 1 vector A_n1)
 *   U        = sum_mu w1_mu tanh(sum_nu W0_{mu nu} s_nu q_nu - b0_mu) - b1
 *
 * Every Y_lm is built at start-up as an explicit polynomial from the
 * Legendre polynomials (Rodrigues' coefficients), its m-th derivative and
 * (x + i y)^m; gradients are exact polynomial derivatives.  3j symbols use
 * the Racah formula.  Neighbours are found by brute force over all pairs
 * with the minimum-image convention (orthorhombic cells).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_LMAX 4
#define OR_NMAX 16 /* max radial functions per set */
#define OR_KMAX 16 /* max Chebyshev terms */
#define OR_HMAX 256
#define OR_DMAX 256

enum { OR_OK = 0, OR_E_INVALID = -1, OR_E_SPECIES = -2, OR_E_BOX = -3,
       OR_E_OVERLAP = -4, OR_E_NONFINITE = -5, OR_E_CAP = -9 };

/* Model as seen by the oracle (own definition; mirrors the paper's notions). */
typedef struct {
    int32_t kind;       /* 1 = dipole (tensor head only), 2 = polarizability (tensor + scalar head),
                           3 = potential-energy surface (one head: the site energy) */
    int32_t n_species;
    double rc_radial, rc_angular;
    int32_t n_max_radial, n_max_angular; /* number of functions = n_max + 1 */
    int32_t basis_radial, basis_angular; /* number of Chebyshev terms = basis + 1 */
    int32_t l_max;
    int32_t four_body;
    int32_t n_hidden;
    const double* c_radial;   /* [T][T][n_R+1][K_R+1] indexed by (t_i, t_j) */
    const double* c_angular;  /* [T][T][n_A+1][K_A+1] */
    const double* q_scaler;   /* [D] */
    const double* w0[2];      /* head 0 = tensor head, head 1 = scalar head; [H][D] */
    const double* b0[2];      /* [H] */
    const double* w1[2];      /* [H] */
    double b1[2];
    int32_t per_species;         /* 1: one network per centre species: w0 [T][H][D], b0 and
                                    w1 [T][H], output biases b1_species[head] [T] */
    const double* b1_species[2];
    int32_t five_body;           /* 1: the l = 1 five-body invariants q5_n (after q4) */
} or_model;

/* ------------------------------------------------------------------------ */
/* Real orthonormal spherical harmonics as explicit polynomials.            */
/* poly[l][m + l][a][b][c] is the coefficient of x^a y^b z^c in r^l Y_lm.   */

static double g_poly[OR_LMAX + 1][2 * OR_LMAX + 1][OR_LMAX + 1][OR_LMAX + 1][OR_LMAX + 1];
static int g_ready = 0;

static double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}
static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

static void build_poly(void) {
    memset(g_poly, 0, sizeof(g_poly));
    for (int l = 0; l <= OR_LMAX; ++l) {
        /* Legendre P_l(t) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) t^(l-2k) */
        double leg[OR_LMAX + 1] = {0};
        for (int k = 0; 2 * k <= l; ++k)
            leg[l - 2 * k] = pow(-1.0, k) * binom(l, k) * binom(2 * l - 2 * k, l) / pow(2.0, l);
        for (int m = 0; m <= l; ++m) {
            /* d^m P_l / dt^m */
            double der[OR_LMAX + 1] = {0};
            for (int q = m; q <= l; ++q) der[q - m] = leg[q] * fact(q) / fact(q - m);
            /* Z(x,y,z) = sum_p der[p] z^p (x^2+y^2+z^2)^((l-m-p)/2) */
            double Z[OR_LMAX + 1][OR_LMAX + 1][OR_LMAX + 1];
            memset(Z, 0, sizeof(Z));
            for (int p = 0; p <= l - m; ++p) {
                if (der[p] == 0.0) continue;
                int s2 = l - m - p;
                if (s2 % 2) continue; /* parity: such coefficients are zero anyway */
                int s = s2 / 2;
                for (int i = 0; i <= s; ++i)
                    for (int j = 0; i + j <= s; ++j) {
                        int k = s - i - j;
                        double mult = fact(s) / (fact(i) * fact(j) * fact(k));
                        Z[2 * i][2 * j][2 * k + p] += der[p] * mult;
                    }
            }
            /* (x + i y)^m = sum_k C(m,k) x^(m-k) (i y)^k */
            double re[OR_LMAX + 1][OR_LMAX + 1], im[OR_LMAX + 1][OR_LMAX + 1];
            memset(re, 0, sizeof(re));
            memset(im, 0, sizeof(im));
            for (int k = 0; k <= m; ++k) {
                double c = binom(m, k);
                int r4 = k % 4; /* i^k = 1, i, -1, -i */
                if (r4 == 0) re[m - k][k] += c;
                if (r4 == 1) im[m - k][k] += c;
                if (r4 == 2) re[m - k][k] -= c;
                if (r4 == 3) im[m - k][k] -= c;
            }
            double nlm = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * fact(l - m) / fact(l + m));
            for (int a1 = 0; a1 <= m; ++a1)
                for (int b1 = 0; a1 + b1 <= m; ++b1) {
                    if (re[a1][b1] == 0.0 && im[a1][b1] == 0.0) continue;
                    for (int a2 = 0; a2 <= l; ++a2)
                        for (int b2 = 0; b2 <= l; ++b2)
                            for (int c2 = 0; c2 <= l; ++c2) {
                                double z = Z[a2][b2][c2];
                                if (z == 0.0) continue;
                                int a = a1 + a2, b = b1 + b2, c = c2;
                                if (a > OR_LMAX || b > OR_LMAX || c > OR_LMAX) continue;
                                if (m == 0) {
                                    g_poly[l][l][a][b][c] += nlm * re[a1][b1] * z;
                                } else {
                                    g_poly[l][l + m][a][b][c] += sqrt(2.0) * nlm * re[a1][b1] * z;
                                    g_poly[l][l - m][a][b][c] += sqrt(2.0) * nlm * im[a1][b1] * z;
                                }
                            }
                }
        }
    }
}

/* 3j symbol (j1 j2 j3; m1 m2 m3) by the Racah formula. */
double or_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < abs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (abs(m1) > j1 || abs(m2) > j2 || abs(m3) > j3) return 0.0;
    double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
    double pre = sqrt(tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) *
                      fact(j3 + m3) * fact(j3 - m3));
    int kmin = 0;
    if (j2 - j3 - m1 > kmin) kmin = j2 - j3 - m1;
    if (j1 - j3 + m2 > kmin) kmin = j1 - j3 + m2;
    int kmax = j1 + j2 - j3;
    if (j1 - m1 < kmax) kmax = j1 - m1;
    if (j2 + m2 < kmax) kmax = j2 + m2;
    double s = 0.0;
    for (int k = kmin; k <= kmax; ++k) {
        double den = fact(k) * fact(j1 + j2 - j3 - k) * fact(j1 - m1 - k) * fact(j2 + m2 - k) *
                     fact(j3 - j2 + m1 + k) * fact(j3 - j1 - m2 + k);
        s += ((k % 2) ? -1.0 : 1.0) / den;
    }
    double sign = ((j1 - j2 - m3) % 2 != 0) ? -1.0 : 1.0;
    return sign * pre * s;
}

void or_init(void) {
    if (g_ready) return;
    build_poly();
    g_ready = 1;
}

/* Threads of the frame loops (OpenMP); for timing the oracle on one core. */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_max_threads(void) { return omp_get_max_threads(); }

/* Y_lm(r/|r|) and its gradient with respect to the vector r.
 * With P = r^l Y_lm (homogeneous of degree l): Y = P(r)/r^l,
 * grad Y = grad P / r^l - l P r / r^(l+2). */
double or_ylm(int l, int m, const double v[3], double grad[3]) {
    or_init();
    double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double r = sqrt(r2);
    double px[OR_LMAX + 1], py[OR_LMAX + 1], pz[OR_LMAX + 1];
    px[0] = py[0] = pz[0] = 1.0;
    for (int k = 1; k <= OR_LMAX; ++k) {
        px[k] = px[k - 1] * v[0];
        py[k] = py[k - 1] * v[1];
        pz[k] = pz[k - 1] * v[2];
    }
    double P = 0.0, dP[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a <= l; ++a)
        for (int b = 0; a + b <= l; ++b) {
            int c = l - a - b;
            double co = g_poly[l][l + m][a][b][c];
            if (co == 0.0) continue;
            P += co * px[a] * py[b] * pz[c];
            if (a > 0) dP[0] += co * a * px[a - 1] * py[b] * pz[c];
            if (b > 0) dP[1] += co * b * px[a] * py[b - 1] * pz[c];
            if (c > 0) dP[2] += co * c * px[a] * py[b] * pz[c - 1];
        }
    double rl = pow(r, l);
    if (grad) {
        for (int d = 0; d < 3; ++d) grad[d] = dP[d] / rl - l * P * v[d] / (rl * r2);
    }
    return P / rl;
}

/* ------------------------------------------------------------------------ */
/* Cutoff and Chebyshev radial basis.                                       */

void or_cutoff(double r, double rc, double* fc, double* dfc) {
    if (r >= rc) {
        *fc = 0.0;
        *dfc = 0.0;
        return;
    }
    *fc = 0.5 * (1.0 + cos(M_PI * r / rc));
    *dfc = -0.5 * M_PI / rc * sin(M_PI * r / rc);
}

/* f_k(r) = (T_k(x)+1)/2 f_c(r) and d f_k / dr, k = 0..K. */
void or_basis(double r, double rc, int K, double* f, double* df) {
    double fc, dfc;
    or_cutoff(r, rc, &fc, &dfc);
    double t = r / rc - 1.0;
    double x = 2.0 * t * t - 1.0;
    double dx = 4.0 * t / rc;
    double T[OR_KMAX + 1], dT[OR_KMAX + 1]; /* T_k(x) and dT_k/dx */
    T[0] = 1.0;
    dT[0] = 0.0;
    if (K >= 1) {
        T[1] = x;
        dT[1] = 1.0;
    }
    for (int k = 1; k < K; ++k) {
        T[k + 1] = 2.0 * x * T[k] - T[k - 1];
        dT[k + 1] = 2.0 * T[k] + 2.0 * x * dT[k] - dT[k - 1];
    }
    for (int k = 0; k <= K; ++k) {
        f[k] = 0.5 * (T[k] + 1.0) * fc;
        df[k] = 0.5 * dT[k] * dx * fc + 0.5 * (T[k] + 1.0) * dfc;
    }
}

/* g_n(r) and g_n'(r) for one coefficient block c[n][k]. */
static void radial_functions(double r, double rc, int nmax, int K, const double* c, double* g,
                             double* dg) {
    double f[OR_KMAX + 1], df[OR_KMAX + 1];
    or_basis(r, rc, K, f, df);
    for (int n = 0; n <= nmax; ++n) {
        double s = 0.0, ds = 0.0;
        for (int k = 0; k <= K; ++k) {
            s += c[n * (K + 1) + k] * f[k];
            ds += c[n * (K + 1) + k] * df[k];
        }
        g[n] = s;
        dg[n] = ds;
    }
}

int or_descriptor_size(const or_model* m) {
    return (m->n_max_radial + 1) + (m->n_max_angular + 1) * m->l_max +
           (m->four_body ? (m->n_max_angular + 1) : 0) + (m->five_body ? (m->n_max_angular + 1) : 0);
}

/* Map the real l=2 sums A[m+2] to complex Condon-Shortley sums At[m+2].
 * For m > 0: Y_l^m = (-1)^m (Y_{l,m} + i Y_{l,-m}) / sqrt2,
 *            Y_l^-m = (Y_{l,m} - i Y_{l,-m}) / sqrt2, Y_l^0 = Y_{l,0}. */
static void real_to_complex_l2(const double* A, double* re, double* im) {
    const double h = 1.0 / sqrt(2.0);
    re[2] = A[2];
    im[2] = 0.0;
    for (int m = 1; m <= 2; ++m) {
        double s = (m % 2) ? -1.0 : 1.0;
        re[2 + m] = s * h * A[2 + m];
        im[2 + m] = s * h * A[2 - m];
        re[2 - m] = h * A[2 + m];
        im[2 - m] = -h * A[2 - m];
    }
}

/* q4 = sum 3j At At At (real part) and dq4/dA (real A, 5 comps), by
 * complex-linear chain rule through the map above. */
static double four_body(const double* A, double* dq_dA) {
    double re[5], im[5];
    real_to_complex_l2(A, re, im);
    double qre = 0.0, qim = 0.0;
    double gre[5] = {0}, gim[5] = {0}; /* dq/dAt_m (holomorphic derivative) */
    for (int m1 = -2; m1 <= 2; ++m1)
        for (int m2 = -2; m2 <= 2; ++m2) {
            int m3 = -m1 - m2;
            if (m3 < -2 || m3 > 2) continue;
            double w = or_wigner3j(2, 2, 2, m1, m2, m3);
            if (w == 0.0) continue;
            int i1 = m1 + 2, i2 = m2 + 2, i3 = m3 + 2;
            /* product of three complex numbers */
            double pr = re[i1] * re[i2] - im[i1] * im[i2];
            double pi = re[i1] * im[i2] + im[i1] * re[i2];
            qre += w * (pr * re[i3] - pi * im[i3]);
            qim += w * (pr * im[i3] + pi * re[i3]);
            /* d/dAt_{m1} of the term = w At_m2 At_m3; sum over all slots gives 3x by symmetry,
             * but accumulate each slot explicitly instead of relying on it. */
            double a23r = re[i2] * re[i3] - im[i2] * im[i3], a23i = re[i2] * im[i3] + im[i2] * re[i3];
            double a13r = re[i1] * re[i3] - im[i1] * im[i3], a13i = re[i1] * im[i3] + im[i1] * re[i3];
            gre[i1] += w * a23r;
            gim[i1] += w * a23i;
            gre[i2] += w * a13r;
            gim[i2] += w * a13i;
            gre[i3] += w * pr;
            gim[i3] += w * pi;
        }
    (void)qim;
    if (dq_dA) {
        /* dAt_m/dA_k for the map above; dq/dA_k = Re(sum_m g_m dAt_m/dA_k) */
        const double h = 1.0 / sqrt(2.0);
        for (int k = 0; k < 5; ++k) dq_dA[k] = 0.0;
        dq_dA[2] += gre[2];
        for (int m = 1; m <= 2; ++m) {
            double s = (m % 2) ? -1.0 : 1.0;
            /* At_{+m} = s h (A_{+m} + i A_{-m}) */
            dq_dA[2 + m] += s * h * gre[2 + m];
            dq_dA[2 - m] += -s * h * gim[2 + m]; /* Re(g * i) = -Im(g) */
            /* At_{-m} = h (A_{+m} - i A_{-m}) */
            dq_dA[2 + m] += h * gre[2 - m];
            dq_dA[2 - m] += h * gim[2 - m]; /* Re(g * (-i)) = Im(g) */
        }
    }
    return qre;
}

/* Imaginary part of the 4-body sum, exposed so tests can check it vanishes. */
double or_four_body_imag(const double* A) {
    double re[5], im[5];
    real_to_complex_l2(A, re, im);
    double qim = 0.0;
    for (int m1 = -2; m1 <= 2; ++m1)
        for (int m2 = -2; m2 <= 2; ++m2) {
            int m3 = -m1 - m2;
            if (m3 < -2 || m3 > 2) continue;
            double w = or_wigner3j(2, 2, 2, m1, m2, m3);
            int i1 = m1 + 2, i2 = m2 + 2, i3 = m3 + 2;
            double pr = re[i1] * re[i2] - im[i1] * im[i2];
            double pi = re[i1] * im[i2] + im[i1] * re[i2];
            qim += w * (pr * im[i3] + pi * re[i3]);
        }
    return qim;
}

double or_four_body(const double* A, double* dq_dA) { return four_body(A, dq_dA); }

/* ------------------------------------------------------------------------ */
/* One atom: descriptor, network, partial forces.                           */

#define OR_LM ((OR_LMAX + 1) * (OR_LMAX + 1))

/* Evaluate head `head` for atom i of species ti with n neighbours given by
 * pair vectors vec[j] = r_j - r_i (all within rc_radial) of species tj[j].
 * Outputs (each may be NULL): U, q[D], dUdq[D], dUdr[n][3].
 * Returns OR_OK or an error code. */
int or_atom_eval(const or_model* mdl, int head, int ti, int n, const double* vec, const int32_t* tj,
                 double* U_out, double* q_out, double* dUdq_out, double* dUdr) {
    or_init();
    const int T = mdl->n_species;
    const int nR = mdl->n_max_radial, nA = mdl->n_max_angular;
    const int KR = mdl->basis_radial, KA = mdl->basis_angular;
    const int lmax = mdl->l_max, H = mdl->n_hidden;
    const int D = or_descriptor_size(mdl);
    if (ti < 0 || ti >= T) return OR_E_SPECIES;
    if (nR + 1 > OR_NMAX || nA + 1 > OR_NMAX || KR > OR_KMAX || KA > OR_KMAX) return OR_E_INVALID;
    if (lmax < 1 || lmax > OR_LMAX || H > OR_HMAX || D > OR_DMAX) return OR_E_INVALID;
    if (mdl->four_body && lmax < 2) return OR_E_INVALID;
    if (head < 0 || head > 1 || (head == 1 && mdl->kind != 2)) return OR_E_INVALID;

    double q[OR_DMAX];
    double A[OR_NMAX][OR_LM];
    memset(q, 0, sizeof(q));
    memset(A, 0, sizeof(A));
    /* forward pass over neighbours */
    for (int j = 0; j < n; ++j) {
        if (tj[j] < 0 || tj[j] >= T) return OR_E_SPECIES;
        const double* v = vec + 3 * j;
        double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (!(r > 1e-8)) return OR_E_OVERLAP;
        double g[OR_NMAX], dg[OR_NMAX];
        if (r < mdl->rc_radial) {
            const double* c = mdl->c_radial + (size_t)(ti * T + tj[j]) * (nR + 1) * (KR + 1);
            radial_functions(r, mdl->rc_radial, nR, KR, c, g, dg);
            for (int k = 0; k <= nR; ++k) q[k] += g[k];
        }
        if (r < mdl->rc_angular) {
            const double* c = mdl->c_angular + (size_t)(ti * T + tj[j]) * (nA + 1) * (KA + 1);
            radial_functions(r, mdl->rc_angular, nA, KA, c, g, dg);
            for (int l = 1; l <= lmax; ++l)
                for (int m = -l; m <= l; ++m) {
                    double Y = or_ylm(l, m, v, NULL);
                    for (int k = 0; k <= nA; ++k) A[k][l * l + l + m] += g[k] * Y;
                }
        }
    }
    /* angular invariants */
    int off = nR + 1;
    for (int l = 1; l <= lmax; ++l)
        for (int k = 0; k <= nA; ++k) {
            double s = 0.0;
            for (int m = -l; m <= l; ++m) s += A[k][l * l + l + m] * A[k][l * l + l + m];
            q[off + (l - 1) * (nA + 1) + k] = s;
        }
    double d4[OR_NMAX][5];
    if (mdl->four_body) {
        int off4 = nR + 1 + lmax * (nA + 1);
        for (int k = 0; k <= nA; ++k) q[off4 + k] = four_body(&A[k][4], d4[k]);
    }
    /* five-body: the one degree-4 rotation invariant of the l = 1 vector
     * A_n1 = (A_n1m)_m, its squared norm squared: q5_n = (sum_m A_n1m^2)^2 */
    const int off5 = nR + 1 + lmax * (nA + 1) + (mdl->four_body ? nA + 1 : 0);
    if (mdl->five_body) {
        for (int k = 0; k <= nA; ++k) {
            double s = 0.0;
            for (int m = -1; m <= 1; ++m) s += A[k][2 + m] * A[k][2 + m];
            q[off5 + k] = s * s;
        }
    }
    if (q_out) memcpy(q_out, q, sizeof(double) * D);

    /* network (the centre species' own network when per_species is set) */
    const size_t sp = mdl->per_species ? (size_t)ti : 0;
    const double* W0 = mdl->w0[head] + sp * H * D;
    const double* b0 = mdl->b0[head] + sp * H;
    const double* w1 = mdl->w1[head] + sp * H;
    double h[OR_HMAX];
    double U = -(mdl->per_species ? mdl->b1_species[head][ti] : mdl->b1[head]);
    for (int mu = 0; mu < H; ++mu) {
        double x = -b0[mu];
        for (int nu = 0; nu < D; ++nu) x += W0[mu * D + nu] * mdl->q_scaler[nu] * q[nu];
        h[mu] = tanh(x);
        U += w1[mu] * h[mu];
    }
    if (U_out) *U_out = U;
    double dUdq[OR_DMAX];
    for (int nu = 0; nu < D; ++nu) {
        double s = 0.0;
        for (int mu = 0; mu < H; ++mu) s += w1[mu] * (1.0 - h[mu] * h[mu]) * W0[mu * D + nu];
        dUdq[nu] = s * mdl->q_scaler[nu];
    }
    if (dUdq_out) memcpy(dUdq_out, dUdq, sizeof(double) * D);
    if (!dUdr) return OR_OK;

    /* dU/dA_nlm */
    double G[OR_NMAX][OR_LM];
    memset(G, 0, sizeof(G));
    for (int l = 1; l <= lmax; ++l)
        for (int k = 0; k <= nA; ++k) {
            double dq = dUdq[off + (l - 1) * (nA + 1) + k];
            for (int m = -l; m <= l; ++m) G[k][l * l + l + m] = 2.0 * dq * A[k][l * l + l + m];
        }
    if (mdl->four_body) {
        int off4 = nR + 1 + lmax * (nA + 1);
        for (int k = 0; k <= nA; ++k)
            for (int mm = 0; mm < 5; ++mm) G[k][4 + mm] += dUdq[off4 + k] * d4[k][mm];
    }
    if (mdl->five_body) {
        /* d q5 / d A_n1m = 2 (sum_m' A_n1m'^2) * 2 A_n1m */
        for (int k = 0; k <= nA; ++k) {
            double s = 0.0;
            for (int m = -1; m <= 1; ++m) s += A[k][2 + m] * A[k][2 + m];
            for (int m = -1; m <= 1; ++m) G[k][2 + m] += dUdq[off5 + k] * 4.0 * s * A[k][2 + m];
        }
    }
    /* backward pass over neighbours: partial forces */
    for (int j = 0; j < n; ++j) {
        const double* v = vec + 3 * j;
        double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        double u[3] = {v[0] / r, v[1] / r, v[2] / r};
        double F[3] = {0.0, 0.0, 0.0};
        double g[OR_NMAX], dg[OR_NMAX];
        if (r < mdl->rc_radial) {
            const double* c = mdl->c_radial + (size_t)(ti * T + tj[j]) * (nR + 1) * (KR + 1);
            radial_functions(r, mdl->rc_radial, nR, KR, c, g, dg);
            double s = 0.0;
            for (int k = 0; k <= nR; ++k) s += dUdq[k] * dg[k];
            for (int d = 0; d < 3; ++d) F[d] += s * u[d];
        }
        if (r < mdl->rc_angular) {
            const double* c = mdl->c_angular + (size_t)(ti * T + tj[j]) * (nA + 1) * (KA + 1);
            radial_functions(r, mdl->rc_angular, nA, KA, c, g, dg);
            for (int l = 1; l <= lmax; ++l)
                for (int m = -l; m <= l; ++m) {
                    double gy[3];
                    double Y = or_ylm(l, m, v, gy);
                    for (int k = 0; k <= nA; ++k) {
                        double Gk = G[k][l * l + l + m];
                        for (int d = 0; d < 3; ++d) F[d] += Gk * (dg[k] * Y * u[d] + g[k] * gy[d]);
                    }
                }
        }
        for (int d = 0; d < 3; ++d) dUdr[3 * j + d] = F[d];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Neighbour search (brute force, minimum image).                           */

/* Simulation box of one frame: periodic flags, and either the orthorhombic
 * edges L or (triclinic) the lattice vectors as the rows of H with the inverse
 * Hinv (Cramer's rule). */
typedef struct {
    int per[3];
    int tric;
    double L[3];
    double H[9], Hinv[9];
} or_box;

static int frame_box(const double* cell, const uint8_t* pbc, double rc, or_box* b) {
    memset(b, 0, sizeof(*b));
    for (int d = 0; d < 3; ++d) b->per[d] = pbc ? (pbc[d] != 0) : 0;
    if (!pbc) return OR_OK;
    if (!cell) {
        for (int d = 0; d < 3; ++d)
            if (b->per[d]) return OR_E_BOX;
        return OR_OK;
    }
    int skew = 0;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            if (a != c && cell[3 * a + c] != 0.0 && (b->per[a] || b->per[c])) skew = 1;
    if (!skew) {
        for (int d = 0; d < 3; ++d) {
            b->L[d] = cell[4 * d];
            if (b->per[d] && !(b->L[d] >= 2.0 * rc)) return OR_E_BOX;
        }
        return OR_OK;
    }
    /* triclinic: all axes periodic, every face-to-face width >= 2 rc */
    if (!(b->per[0] && b->per[1] && b->per[2])) return OR_E_BOX;
    b->tric = 1;
    memcpy(b->H, cell, sizeof(b->H));
    const double* h = cell;
    double cof[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            cof[3 * i + j] = h[3 * i1 + j1] * h[3 * i2 + j2] - h[3 * i1 + j2] * h[3 * i2 + j1];
        }
    const double det = h[0] * cof[0] + h[1] * cof[1] + h[2] * cof[2];
    if (!(fabs(det) > 0.0)) return OR_E_BOX;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) b->Hinv[3 * i + j] = cof[3 * j + i] / det;
    for (int k = 0; k < 3; ++k) {
        /* width along k: |det| / |h_{k+1} x h_{k+2}| = |det| / |cofactor row k| */
        const double n = sqrt(cof[3 * k] * cof[3 * k] + cof[3 * k + 1] * cof[3 * k + 1] + cof[3 * k + 2] * cof[3 * k + 2]);
        if (!(fabs(det) / n >= 2.0 * rc)) return OR_E_BOX;
    }
    return OR_OK;
}

/* r_j - r_i under the minimum-image convention.  Triclinic: the difference is
 * first brought into the unit cell in fractional coordinates s = d Hinv, then
 * the shortest of the images s + n, n in {-2..1}^3, is taken. */
static void pair_vector(const double* pi, const double* pj, const or_box* b, double v[3]) {
    if (!b->tric) {
        for (int d = 0; d < 3; ++d) {
            double x = pj[d] - pi[d];
            if (b->per[d]) x -= b->L[d] * nearbyint(x / b->L[d]);
            v[d] = x;
        }
        return;
    }
    double d0[3], f[3];
    for (int d = 0; d < 3; ++d) d0[d] = pj[d] - pi[d];
    for (int k = 0; k < 3; ++k) {
        f[k] = d0[0] * b->Hinv[k] + d0[1] * b->Hinv[3 + k] + d0[2] * b->Hinv[6 + k];
        f[k] -= floor(f[k]);
    }
    double best = INFINITY;
    for (int n0 = -2; n0 <= 1; ++n0)
        for (int n1 = -2; n1 <= 1; ++n1)
            for (int n2 = -2; n2 <= 1; ++n2) {
                const double g[3] = {f[0] + n0, f[1] + n1, f[2] + n2};
                double w[3];
                for (int d = 0; d < 3; ++d) w[d] = g[0] * b->H[d] + g[1] * b->H[3 + d] + g[2] * b->H[6 + d];
                const double r2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
                if (r2 < best) {
                    best = r2;
                    memcpy(v, w, sizeof(w));
                }
            }
}

/* For each atom i (0..n-1) write the neighbours j != i with |r_ij| < rc into
 * list[i*cap ...] in increasing j order; count[i] receives their number.
 * Returns OR_E_CAP if any atom has more than cap neighbours. */
int or_neighbors(int n, const double* pos, const double* cell, const uint8_t* pbc, double rc,
                 int cap, int32_t* count, int32_t* list) {
    or_box box;
    int e = frame_box(cell, pbc, rc, &box);
    if (e) return e;
    int overflow = 0;
    for (int i = 0; i < n; ++i) {
        int c = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double v[3];
            pair_vector(pos + 3 * i, pos + 3 * j, &box, v);
            double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            if (r2 < rc * rc) {
                if (c < cap) list[(size_t)i * cap + c] = j;
                ++c;
            }
        }
        count[i] = c;
        if (c > cap) overflow = 1;
    }
    return overflow ? OR_E_CAP : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole frames: mu (kind 1, 3 values) or alpha (kind 2, 9 values).          */

static int eval_atom_tensor(const or_model* mdl, int n_at, const double* pos, const int32_t* spc,
                            const or_box* box, int i, double* t_out) {
    /* gather neighbours within rc_radial */
    const double rc = mdl->rc_radial;
    int cap = 64, n = 0;
    double* vec = (double*)malloc(sizeof(double) * 3 * cap);
    int32_t* tj = (int32_t*)malloc(sizeof(int32_t) * cap);
    for (int j = 0; j < n_at; ++j) {
        if (j == i) continue;
        double v[3];
        pair_vector(pos + 3 * i, pos + 3 * j, box, v);
        if (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] < rc * rc) {
            if (n == cap) {
                cap *= 2;
                vec = (double*)realloc(vec, sizeof(double) * 3 * cap);
                tj = (int32_t*)realloc(tj, sizeof(int32_t) * cap);
            }
            memcpy(vec + 3 * n, v, sizeof(v));
            tj[n] = spc[j];
            ++n;
        }
    }
    double* F = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    double Ut = 0.0, Us = 0.0;
    int e = or_atom_eval(mdl, 0, spc[i], n, vec, tj, &Ut, NULL, NULL, F);
    if (!e && mdl->kind == 2) e = or_atom_eval(mdl, 1, spc[i], n, vec, tj, &Us, NULL, NULL, NULL);
    if (!e) {
        if (mdl->kind == 1) {
            double mu[3] = {0, 0, 0};
            for (int j = 0; j < n; ++j) {
                const double* v = vec + 3 * j;
                double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                for (int d = 0; d < 3; ++d) mu[d] -= r2 * F[3 * j + d];
            }
            memcpy(t_out, mu, sizeof(mu));
        } else {
            double a[9] = {0};
            for (int j = 0; j < n; ++j)
                for (int u = 0; u < 3; ++u)
                    for (int w = 0; w < 3; ++w) a[3 * u + w] -= vec[3 * j + u] * F[3 * j + w];
            for (int d = 0; d < 3; ++d) a[4 * d] += Us;
            memcpy(t_out, a, sizeof(a));
        }
    }
    free(vec);
    free(tj);
    free(F);
    return e;
}

/* Evaluate n_frames frames stored CSR-style (atom_offsets[n_frames+1]).
 * out: [n_frames][3] (dipole) or [n_frames][9] (polarizability), per_atom
 * (optional) the same per atom.  cells/pbc may be NULL (vacuum). */
int or_eval_frames(const or_model* mdl, int n_frames, const int64_t* atom_offsets, const double* pos,
                   const int32_t* species, const double* cells, const uint8_t* pbc, double* out,
                   double* per_atom) {
    or_init();
    if (mdl->kind != 1 && mdl->kind != 2) return OR_E_INVALID;
    const int nt = (mdl->kind == 1) ? 3 : 9;
    for (int f = 0; f < n_frames; ++f) {
        const int64_t a0 = atom_offsets[f], a1 = atom_offsets[f + 1];
        const int n_at = (int)(a1 - a0);
        or_box box;
        int e = frame_box(cells ? cells + 9 * f : NULL, pbc ? pbc + 3 * f : NULL, mdl->rc_radial, &box);
        if (e) return e;
        for (int64_t a = a0; a < a1; ++a)
            for (int d = 0; d < 3; ++d)
                if (!isfinite(pos[3 * a + d])) return OR_E_NONFINITE;
        double* tens = (double*)malloc(sizeof(double) * nt * (n_at > 0 ? n_at : 1));
        int err = 0;
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n_at; ++i) {
            int ei = eval_atom_tensor(mdl, n_at, pos + 3 * a0, species + a0, &box, i, tens + nt * i);
            if (ei) {
#pragma omp critical
                err = ei;
            }
        }
        if (err) {
            free(tens);
            return err;
        }
        for (int k = 0; k < nt; ++k) {
            double s = 0.0;
            for (int i = 0; i < n_at; ++i) s += tens[nt * i + k];
            out[(size_t)f * nt + k] = s;
        }
        if (per_atom) memcpy(per_atom + (size_t)a0 * nt, tens, sizeof(double) * nt * n_at);
        free(tens);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Potential-energy surface (kind 3): per frame U = sum_i U_i (Sec. 2.1, Eq.  */
/* site-energy), W = -sum_i sum_j r_ij (x) dU_i/dr_ij (Sec. 2.1, Eq. virial)  */
/* and forces F_k = -dU/dr_k.  With r_ij = r_j - r_i, dr_ij/dr_k is +1 for    */
/* j = k and -1 for i = k, so atom i gets +dU_i/dr_ij and atom j gets          */
/* -dU_i/dr_ij from every pair (i, j).                                         */

typedef struct {
    int n;
    int32_t* j;   /* frame-local neighbour index */
    double* dudr; /* [n][3] dU_i/dr_ij */
} pes_pairs;

int or_eval_pes(const or_model* mdl, int n_frames, const int64_t* atom_offsets, const double* pos,
                const int32_t* species, const double* cells, const uint8_t* pbc, double* energy, double* virial,
                double* forces, double* per_atom_energy) {
    or_init();
    if (mdl->kind != 3) return OR_E_INVALID;
    for (int f = 0; f < n_frames; ++f) {
        const int64_t a0 = atom_offsets[f], a1 = atom_offsets[f + 1];
        const int n_at = (int)(a1 - a0);
        or_box box;
        int e = frame_box(cells ? cells + 9 * f : NULL, pbc ? pbc + 3 * f : NULL, mdl->rc_radial, &box);
        if (e) return e;
        for (int64_t a = a0; a < a1; ++a)
            for (int d = 0; d < 3; ++d)
                if (!isfinite(pos[3 * a + d])) return OR_E_NONFINITE;
        const double* p = pos + 3 * a0;
        const int32_t* spc = species + a0;
        const int nn = n_at > 0 ? n_at : 1;
        double* U = (double*)malloc(sizeof(double) * nn);
        double* W = (double*)malloc(sizeof(double) * 9 * nn);
        pes_pairs* pairs = (pes_pairs*)calloc((size_t)nn, sizeof(pes_pairs));
        int err = 0;
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n_at; ++i) {
            const double rc = mdl->rc_radial;
            int n = 0;
            for (int j = 0; j < n_at; ++j) {
                if (j == i) continue;
                double v[3];
                pair_vector(p + 3 * i, p + 3 * j, &box, v);
                if (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] < rc * rc) ++n;
            }
            double* vec = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
            int32_t* tj = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
            int32_t* jj = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
            double* dudr = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
            int k = 0;
            for (int j = 0; j < n_at; ++j) {
                if (j == i) continue;
                double v[3];
                pair_vector(p + 3 * i, p + 3 * j, &box, v);
                if (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] < rc * rc) {
                    memcpy(vec + 3 * k, v, sizeof(v));
                    tj[k] = spc[j];
                    jj[k] = j;
                    ++k;
                }
            }
            int ei = or_atom_eval(mdl, 0, spc[i], n, vec, tj, &U[i], NULL, NULL, dudr);
            for (int c = 0; c < 9; ++c) W[9 * i + c] = 0.0;
            for (int q = 0; q < n && !ei; ++q)
                for (int u = 0; u < 3; ++u)
                    for (int w = 0; w < 3; ++w) W[9 * i + 3 * u + w] -= vec[3 * q + u] * dudr[3 * q + w];
            pairs[i].n = n;
            pairs[i].j = jj;
            pairs[i].dudr = dudr;
            free(vec);
            free(tj);
            if (ei) {
#pragma omp critical
                err = ei;
            }
        }
        if (!err) {
            double* F = forces + 3 * a0;
            for (int i = 0; i < 3 * n_at; ++i) F[i] = 0.0;
            for (int i = 0; i < n_at; ++i)
                for (int q = 0; q < pairs[i].n; ++q) {
                    const int j = pairs[i].j[q];
                    for (int d = 0; d < 3; ++d) {
                        F[3 * i + d] += pairs[i].dudr[3 * q + d];
                        F[3 * j + d] -= pairs[i].dudr[3 * q + d];
                    }
                }
            double es = 0.0;
            for (int i = 0; i < n_at; ++i) es += U[i];
            energy[f] = es;
            for (int c = 0; c < 9; ++c) {
                double s = 0.0;
                for (int i = 0; i < n_at; ++i) s += W[9 * i + c];
                virial[(size_t)9 * f + c] = s;
            }
            if (per_atom_energy) memcpy(per_atom_energy + a0, U, sizeof(double) * n_at);
        }
        for (int i = 0; i < n_at; ++i) {
            free(pairs[i].j);
            free(pairs[i].dudr);
        }
        free(pairs);
        free(U);
        free(W);
        if (err) return err;
    }
    return OR_OK;
}

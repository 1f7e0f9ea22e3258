/*
 * CPU FP64 oracle for the time-sliced periodic retarded-time field.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, by the build check, by the smoke
 * check and by the CPU baseline leg of the benchmark. The HIP library never
 * links, includes or calls anything here, and nothing here uses the library.
 *
 * What is computed (Sec. 2.1 Eqs. 9-10, Sec. 2.2 Eq. 11 and algorithm
 * steps 2 and 6):
 *
 *   J_b(x) = sum_k sum_c G_{k,b}((x - c) mod N) * S_k(c)
 *
 *   G_{k,b}(c) = (1/m^3) sum_{subpoints a} sum_{images u}
 *                [T_k <= n < T_{k+1}] * pref * phi_b(rho) / (4 pi rho^2)
 *
 * with rho^2 = n h^2, h = L/(2 m N), and n the exact integer
 *   n = sum_d (2m (c_d + u_d N) + o_{a_d})^2,  o_a = 2a + 1 - m,
 * T_k = (r_k/h)*(r_k/h) in IEEE double (half-open shells [r_k, r_{k+1})).
 * When r_0 = 0 the self pair (c = 0, u = 0) is replaced by the exact cube
 * average of pref*phi/(4 pi r^2), which is finite.
 *
 * Every loop here is the plain definition: a sum over cells, images and
 * subpoints; a naive separable DFT; an O(N^6) brute force. Nothing is
 * blocked or reordered beyond skipping images that lie entirely outside the
 * shells (the paper's "effective horizon", algorithm step 2).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t kind;   /* 0: phi=1; 1: max(0, a e^{-(r/s)^p} - c); 2: Eq. 15 hard cut */
    int32_t pad_;
    double a, s, p, c, cut, prefactor;
} or_atten;

static const double OR_PI = 3.141592653589793238462643383279502884;

/* ---- radial factor (Eq. 15 and its continuous variant) ----------------- */

double or_phi(const or_atten *at, double r)
{
    if (at->kind == 0) return 1.0;
    double v = at->a * exp(-pow(r / at->s, at->p)) - at->c;
    if (at->kind == 1) return v > 0.0 ? v : 0.0;
    return (r <= at->cut) ? v : 0.0;
}

/* Upper end of the support of phi (where the integrand stops). */
static double phi_support_end(const or_atten *at)
{
    if (at->kind == 0) return INFINITY;
    if (at->kind == 2) return at->cut;
    if (at->c <= 0.0) return INFINITY;
    if (at->a <= at->c) return 0.0;
    return at->s * pow(log(at->a / at->c), 1.0 / at->p);
}

/* Tanh-sinh quadrature of a e^{-(r/s)^p} - c over [0, U]. The r^p cusp at
 * r = 0 is an endpoint singularity, which this rule handles. Step halving
 * until two levels agree to 1e-16 relative. */
static double smooth_part(const or_atten *at, double r)
{
    return at->a * exp(-pow(r / at->s, at->p)) - at->c;
}

static double tanh_sinh_0U(const or_atten *at, double U)
{
    if (U <= 0.0) return 0.0;
    double prev = 0.0;
    for (int level = 3; level <= 12; ++level) {
        double hstep = ldexp(1.0, -level);
        double sum = 0.0;
        for (int i = -(int)(4.0 / hstep); i <= (int)(4.0 / hstep); ++i) {
            double t = i * hstep;
            double u = 0.5 * OR_PI * sinh(t);
            /* r = U (1 + tanh u) / 2 = U / (1 + e^{-2u}) */
            double r = U / (1.0 + exp(-2.0 * u));
            double ch = cosh(u);
            double w = 0.5 * OR_PI * cosh(t) / (ch * ch);
            if (!(r > 0.0) || r >= U || w == 0.0) continue;
            sum += w * smooth_part(at, r);
        }
        double est = 0.5 * U * hstep * sum;
        if (level > 3 && fabs(est - prev) <= 1e-15 * fabs(est)) return est;
        prev = est;
    }
    return prev;
}

/* Phi(R) = int_0^R phi(r) dr */
double or_Phi(const or_atten *at, double R)
{
    if (R <= 0.0) return 0.0;
    if (at->kind == 0) return R;
    double U = R;
    double e = phi_support_end(at);
    if (U > e) U = e;
    return tanh_sinh_0U(at, U);
}

/* Shell integral of phi over [r0, r1). */
double or_shell_integral(const or_atten *at, double r0, double r1)
{
    return or_Phi(at, r1) - or_Phi(at, r0);
}

/* Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_n. */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = -z; x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Cube average of pref * phi(r) / (4 pi r^2) over the cell [-l/2, l/2]^3.
 * Splitting the cube into six pyramids with apex at the centre, each face
 * contributes int int (l/2) Phi(R) / (4 pi R^3) dy dz with
 * R = sqrt(l^2/4 + y^2 + z^2); the average is 6/l^3 times one face. The
 * face integrand is smooth (R >= l/2), so a tensor Gauss-Legendre rule on
 * the quarter face [0, l/2]^2 (times 4) converges fast. */
double or_self_cell(const or_atten *at, double l)
{
    enum { NG = 48 };
    double gx[NG], gw[NG];
    gauss_legendre(NG, gx, gw);
    double hl = 0.5 * l;
    double acc = 0.0;
    for (int i = 0; i < NG; ++i) {
        double y = 0.5 * hl * (gx[i] + 1.0);
        for (int j = 0; j < NG; ++j) {
            double z = 0.5 * hl * (gx[j] + 1.0);
            double R = sqrt(hl * hl + y * y + z * z);
            acc += gw[i] * gw[j] * hl * or_Phi(at, R) / (R * R * R);
        }
    }
    acc *= 0.25 * hl * hl;                  /* Jacobian of [-1,1]^2 -> [0,l/2]^2 */
    double face = 4.0 * acc / (4.0 * OR_PI); /* whole face */
    return at->prefactor * 6.0 * face / (l * l * l);
}

/* ---- shell kernel (Eq. 10, algorithm step 2) --------------------------- */

typedef struct {
    int N, K, m;
    double L, l, h;
    const double *radii;
    double T[1025];        /* thresholds T_k = (r_k/h)^2, K+1 entries */
    double rmin, rmax;     /* r_0, r_K */
    int U;                 /* image range |u_d| <= U */
    double self_val;       /* cube average for the self pair when r_0 == 0 */
    or_atten at;
} kern_t;

static int kern_init(kern_t *kp, int N, double L, int K, const double *radii,
                     int m, const or_atten *at)
{
    if (K < 1 || K > 1024) return -1;
    kp->N = N; kp->K = K; kp->m = m; kp->L = L;
    kp->l = L / N;
    kp->h = L / (2.0 * m * N);
    kp->radii = radii;
    for (int k = 0; k <= K; ++k) {
        double q = radii[k] / kp->h;
        kp->T[k] = q * q;
    }
    kp->rmin = radii[0];
    kp->rmax = radii[K];
    kp->U = (int)ceil(radii[K] / L) + 1;
    kp->at = *at;
    kp->self_val = (radii[0] == 0.0) ? or_self_cell(at, kp->l) : 0.0;
    return 0;
}

/* Value of one subpoint at squared half-subcell distance n. */
static double point_value(const kern_t *kp, int64_t n)
{
    double rho = sqrt((double)n) * kp->h;
    return kp->at.prefactor * or_phi(&kp->at, rho) /
           (4.0 * OR_PI * rho * rho) / ((double)kp->m * kp->m * kp->m);
}

/* Shell index of n, or -1 when outside [T_0, T_K). */
static int shell_of(const kern_t *kp, int64_t n)
{
    double dn = (double)n;
    if (dn < kp->T[0] || dn >= kp->T[kp->K]) return -1;
    int lo = 0, hi = kp->K;            /* T[lo] <= dn < T[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (kp->T[mid] <= dn) lo = mid; else hi = mid;
    }
    return lo;
}

/* Add the contributions of displacement d = (d0,d1,d2) (cell units, any
 * integers) to out[k0..k1) (absolute shell indices; out is indexed by k-k0).
 * Self pair handled when d == 0 mod N and r_0 == 0. */
static void kern_accumulate(const kern_t *kp, int d0, int d1, int d2,
                            int k0, int k1, double *out)
{
    const int N = kp->N, m = kp->m, U = kp->U;
    const double l = kp->l;
    int dd[3] = { ((d0 % N) + N) % N, ((d1 % N) + N) % N, ((d2 % N) + N) % N };
    const double lo_r = kp->radii[k0], hi_r = kp->radii[k1];
    for (int u0 = -U; u0 <= U; ++u0)
    for (int u1 = -U; u1 <= U; ++u1)
    for (int u2 = -U; u2 <= U; ++u2) {
        int64_t cx[3] = { dd[0] + (int64_t)u0 * N, dd[1] + (int64_t)u1 * N,
                          dd[2] + (int64_t)u2 * N };
        /* bounding test on the whole cell [c - l/2, c + l/2]^3 */
        double mn2 = 0.0, mx2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double c = (double)cx[a] * l;
            double lo = c - 0.5 * l, hi = c + 0.5 * l;
            double near = (lo > 0.0) ? lo : ((hi < 0.0) ? -hi : 0.0);
            double far = fmax(fabs(lo), fabs(hi));
            mn2 += near * near; mx2 += far * far;
        }
        double margin = 1e-9 * (hi_r + l);
        if (sqrt(mn2) > hi_r + margin) continue;
        if (sqrt(mx2) < lo_r - margin) continue;
        if (kp->rmin == 0.0 && cx[0] == 0 && cx[1] == 0 && cx[2] == 0) {
            if (k0 == 0) out[0] += kp->self_val;
            continue;
        }
        for (int a0 = 0; a0 < m; ++a0)
        for (int a1 = 0; a1 < m; ++a1)
        for (int a2 = 0; a2 < m; ++a2) {
            int64_t q0 = 2 * m * cx[0] + (2 * a0 + 1 - m);
            int64_t q1 = 2 * m * cx[1] + (2 * a1 + 1 - m);
            int64_t q2 = 2 * m * cx[2] + (2 * a2 + 1 - m);
            int64_t n = q0 * q0 + q1 * q1 + q2 * q2;
            int k = shell_of(kp, n);
            if (k < k0 || k >= k1) continue;
            out[k - k0] += point_value(kp, n);
        }
    }
}

/* All K shell values at displacement (d0,d1,d2). */
int or_G_at(int N, double L, int K, const double *radii, int m,
            const or_atten *at, int d0, int d1, int d2, double *outK)
{
    kern_t kp;
    if (kern_init(&kp, N, L, K, radii, m, at)) return -1;
    memset(outK, 0, sizeof(double) * K);
    kern_accumulate(&kp, d0, d1, d2, 0, K, outK);
    return 0;
}

/* Dense kernel G[k][i][j][kx] for all K shells over the full N^3 grid.
 * If conserve != 0, each shell is rescaled so that l^3 sum_c G_k(c) equals
 * the shell integral of phi. */
int or_build_G(int N, double L, int K, const double *radii, int m,
               const or_atten *at, int conserve, double *G)
{
    kern_t kp;
    if (kern_init(&kp, N, L, K, radii, m, at)) return -1;
    const int64_t n3 = (int64_t)N * N * N;
    memset(G, 0, sizeof(double) * n3 * K);
    #pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * K);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t c = 0; c < n3; ++c) {
            int i = (int)(c / ((int64_t)N * N)), j = (int)((c / N) % N), x = (int)(c % N);
            memset(tmp, 0, sizeof(double) * K);
            kern_accumulate(&kp, i, j, x, 0, K, tmp);
            for (int k = 0; k < K; ++k) G[(int64_t)k * n3 + c] = tmp[k];
        }
        free(tmp);
    }
    if (conserve) {
        double l3 = kp.l * kp.l * kp.l;
        for (int k = 0; k < K; ++k) {
            double s = 0.0, comp = 0.0;
            for (int64_t c = 0; c < n3; ++c) {      /* Neumaier sum */
                double v = G[(int64_t)k * n3 + c], t = s + v;
                comp += (fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s;
                s = t;
            }
            s += comp;
            double target = or_shell_integral(at, radii[k], radii[k + 1]);
            double f = (s != 0.0) ? target / (l3 * s) : 0.0;
            for (int64_t c = 0; c < n3; ++c) G[(int64_t)k * n3 + c] *= f;
        }
    }
    return 0;
}

/* ---- route D: direct real-space periodic summation (Eq. 11 summed over
 * slices, algorithm step 6) --------------------------------------------- */

/* Neumaier compensated accumulator */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double v)
{
    double t = a->s + v;
    a->c += (fabs(a->s) >= fabs(v)) ? (a->s - t) + v : (v - t) + a->s;
    a->s = t;
}

/* Dense-kernel version: G is K x N^3 for one band; sources of slice k are
 * src_cell[off[k] .. off[k+1]), src_lum likewise. */
int or_field_direct(int N, int K, const double *G,
                    const int64_t *off, const int64_t *src_cell, const double *src_lum,
                    int64_t n_targets, const int64_t *targets, double *J)
{
    const int64_t n3 = (int64_t)N * N * N;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_targets; ++t) {
        int64_t x = targets[t];
        int xi = (int)(x / ((int64_t)N * N)), xj = (int)((x / N) % N), xk = (int)(x % N);
        nsum acc = { 0.0, 0.0 };
        for (int k = 0; k < K; ++k) {
            const double *Gk = G + (int64_t)k * n3;
            for (int64_t s = off[k]; s < off[k + 1]; ++s) {
                int64_t c = src_cell[s];
                int ci = (int)(c / ((int64_t)N * N)), cj = (int)((c / N) % N), ck = (int)(c % N);
                int di = (xi - ci + N) % N, dj = (xj - cj + N) % N, dk = (xk - ck + N) % N;
                nadd(&acc, src_lum[s] * Gk[((int64_t)di * N + dj) * N + dk]);
            }
        }
        J[t] = acc.s + acc.c;
    }
    return 0;
}

/* Kernel-on-demand version for grids whose dense kernel does not fit: each
 * (target, source) pair evaluates only the shell of the source's slice. */
int or_field_direct_ondemand(int N, double L, int K, const double *radii, int m,
                             const or_atten *at,
                             const int64_t *off, const int64_t *src_cell, const double *src_lum,
                             int64_t n_targets, const int64_t *targets, double *J)
{
    kern_t kp;
    if (kern_init(&kp, N, L, K, radii, m, at)) return -1;
    /* Cheap reject: a displacement whose minimum-image distance exceeds r_K
     * plus a cell diagonal, and r_K < L/2 - l, has no image in any shell. */
    const double diag = sqrt(3.0) * kp.l;
    const int single_image = (radii[K] + diag < 0.5 * L - diag);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < n_targets; ++t) {
        int64_t x = targets[t];
        int xi = (int)(x / ((int64_t)N * N)), xj = (int)((x / N) % N), xk = (int)(x % N);
        nsum acc = { 0.0, 0.0 };
        for (int k = 0; k < K; ++k) {
            double lo = radii[k] - diag, hi = radii[k + 1] + diag;
            for (int64_t s = off[k]; s < off[k + 1]; ++s) {
                int64_t c = src_cell[s];
                int ci = (int)(c / ((int64_t)N * N)), cj = (int)((c / N) % N), ck = (int)(c % N);
                int d[3] = { (xi - ci + N) % N, (xj - cj + N) % N, (xk - ck + N) % N };
                if (single_image) {
                    double r2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        int e = d[a] > N / 2 ? N - d[a] : d[a];
                        r2 += (double)e * e;
                    }
                    double r = sqrt(r2) * kp.l;
                    if (r > hi || r < lo) continue;
                }
                double g = 0.0;
                kern_accumulate(&kp, d[0], d[1], d[2], k, k + 1, &g);
                if (g != 0.0) nadd(&acc, src_lum[s] * g);
            }
        }
        J[t] = acc.s + acc.c;
    }
    return 0;
}

/* Kernel-support version for large grids whose outer radius stays well inside
 * half the box (one periodic image can reach a target): the same sum written
 * over displacements, J_b(x) = sum_k sum_d G_{k,b}(d) S_k((x - d) mod N), where
 * d runs over the cells whose minimum-image distance from the origin lies in
 * [r_k - diag, r_{k+1} + diag] (G_{k,b} vanishes elsewhere: every subpoint of
 * any other cell is farther than half a diagonal from the shell). S_k is
 * the nearest-grid-point deposit of slice k's point list. All nb bands share
 * the sources; J is nb x n_targets, band-major. Returns -2 when the outer
 * radius is too large for a single image. */
int or_field_direct_support(int N, double L, int K, const double *radii, int m, int nb,
                            const or_atten *at,
                            const int64_t *off, const int64_t *src_cell, const double *src_lum,
                            int64_t n_targets, const int64_t *targets, double *J)
{
    if (nb < 1 || nb > 16) return -1;
    kern_t kp[16];
    for (int b = 0; b < nb; ++b)
        if (kern_init(&kp[b], N, L, K, radii, m, &at[b])) return -1;
    const double l = L / N, diag = sqrt(3.0) * l;
    if (!(radii[K] + 2.0 * diag < 0.5 * L)) return -2;
    const int64_t n3 = (int64_t)N * N * N;
    double *S = (double *)malloc(sizeof(double) * n3);
    nsum *acc = (nsum *)calloc((size_t)nb * n_targets, sizeof(nsum));
    if (!S || !acc) { free(S); free(acc); return -3; }
    for (int k = 0; k < K; ++k) {
        if (off[k + 1] == off[k]) continue;
        /* deposit of slice k */
        memset(S, 0, sizeof(double) * n3);
        for (int64_t s = off[k]; s < off[k + 1]; ++s) S[src_cell[s]] += src_lum[s];
        /* displacements that can meet shell k */
        const double lo = radii[k] - diag, hi = radii[k + 1] + diag;
        const int R = (int)ceil(hi / l);
        const int W = 2 * R + 1;
        int64_t cand = (int64_t)W * W * W, nd = 0;
        int32_t *dl = (int32_t *)malloc(sizeof(int32_t) * 3 * cand);
        for (int64_t c = 0; c < cand; ++c) {
            int d0 = (int)(c / ((int64_t)W * W)) - R, d1 = (int)((c / W) % W) - R, d2 = (int)(c % W) - R;
            double r = sqrt((double)d0 * d0 + (double)d1 * d1 + (double)d2 * d2) * l;
            if (r < lo || r > hi) continue;
            dl[3 * nd] = d0; dl[3 * nd + 1] = d1; dl[3 * nd + 2] = d2;
            ++nd;
        }
        /* kernel values there, from the definition */
        double *g = (double *)malloc(sizeof(double) * nb * (nd > 0 ? nd : 1));
        #pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < nd; ++i)
            for (int b = 0; b < nb; ++b) {
                double v = 0.0;
                kern_accumulate(&kp[b], dl[3 * i], dl[3 * i + 1], dl[3 * i + 2], k, k + 1, &v);
                g[(int64_t)b * nd + i] = v;
            }
        #pragma omp parallel for schedule(dynamic, 4)
        for (int64_t t = 0; t < n_targets; ++t) {
            int64_t x = targets[t];
            int xi = (int)(x / ((int64_t)N * N)), xj = (int)((x / N) % N), xk = (int)(x % N);
            for (int b = 0; b < nb; ++b) {
                nsum a = acc[(int64_t)b * n_targets + t];
                const double *gb = g + (int64_t)b * nd;
                for (int64_t i = 0; i < nd; ++i) {
                    if (gb[i] == 0.0) continue;
                    int c0 = ((xi - dl[3 * i]) % N + N) % N;
                    int c1 = ((xj - dl[3 * i + 1]) % N + N) % N;
                    int c2 = ((xk - dl[3 * i + 2]) % N + N) % N;
                    double sv = S[((int64_t)c0 * N + c1) * N + c2];
                    if (sv != 0.0) nadd(&a, gb[i] * sv);
                }
                acc[(int64_t)b * n_targets + t] = a;
            }
        }
        free(g);
        free(dl);
    }
    for (int64_t i = 0; i < (int64_t)nb * n_targets; ++i) J[i] = acc[i].s + acc[i].c;
    free(S);
    free(acc);
    return 0;
}

/* ---- background cosmology (Sec. 2.1 Eqs. 4-5) --------------------------
 * Flat universe of matter and a cosmological constant, OL = 1 - Om,
 * H(a) = H0 sqrt(Om a^-3 + OL). Units: Myr (Julian year), comoving Mpc,
 * c = 299792.458 km/s. Every quantity is its defining integral, evaluated
 * by tanh-sinh quadrature (no closed forms here: the tests compare with them). */

static const double OR_C_KMS = 299792.458;
static const double OR_MPC_KM = 3.0856775814913673e19;
static const double OR_MYR_S = 3.15576e13;

typedef double (*or_fn)(double x, const double *par);

/* tanh-sinh quadrature of f over [lo, hi], levels refined until two agree */
static double tanh_sinh(or_fn f, const double *par, double lo, double hi)
{
    if (!(hi > lo)) return 0.0;
    double prev = 0.0, half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    for (int level = 3; level <= 12; ++level) {
        double hstep = ldexp(1.0, -level), sum = 0.0;
        for (int i = -(int)(4.0 / hstep); i <= (int)(4.0 / hstep); ++i) {
            double t = i * hstep;
            double u = 0.5 * OR_PI * sinh(t);
            double ch = cosh(u);
            double w = 0.5 * OR_PI * cosh(t) / (ch * ch);
            double x = mid + half * tanh(u);
            if (!(x > lo) || !(x < hi) || w == 0.0) continue;
            sum += w * f(x, par);
        }
        double est = half * hstep * sum;
        if (level > 3 && fabs(est - prev) <= 1e-15 * fabs(est)) return est;
        prev = est;
    }
    return prev;
}

/* dt/da = 1 / (a H(a)), in Myr per unit a; par = {Om, OL, H0 [1/Myr]} */
static double dt_da(double a, const double *par)
{
    return 1.0 / (a * par[2] * sqrt(par[0] / (a * a * a) + par[1]));
}

/* c / H(z) in Mpc; par = {Om, OL, c/H0 [Mpc]} */
static double c_over_H(double z, const double *par)
{
    double zp = 1.0 + z;
    return par[2] / sqrt(par[0] * zp * zp * zp + par[1]);
}

/* cosmic time at redshift z (Myr): t = int_0^{1/(1+z)} da / (a H(a)) */
double or_cosmic_time(double h, double om, double z)
{
    double par[3] = { om, 1.0 - om, 100.0 * h / OR_MPC_KM * OR_MYR_S };
    return tanh_sinh(dt_da, par, 0.0, 1.0 / (1.0 + z));
}

/* comoving distance between z1 <= z2 (Mpc): int_{z1}^{z2} c dz / H(z) */
double or_comoving_distance(double h, double om, double z1, double z2)
{
    double par[3] = { om, 1.0 - om, OR_C_KMS / (100.0 * h) };
    return tanh_sinh(c_over_H, par, z1, z2);
}

/* redshift at cosmic time t (Myr), by bisection on the monotone t(z) */
double or_redshift_at_time(double h, double om, double t)
{
    double lo = 0.0, hi = 1.0;
    while (or_cosmic_time(h, om, hi) > t) hi *= 2.0;      /* t decreases with z */
    if (or_cosmic_time(h, om, lo) < t) return -1.0;        /* later than z = 0 */
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
        double m = 0.5 * (lo + hi);
        if (or_cosmic_time(h, om, m) > t) lo = m; else hi = m;
    }
    return 0.5 * (lo + hi);
}

/* Dense kernel with one radial factor per slice: G[k] uses at[k] (the
 * self cell of slice 0 with at[0]). */
int or_build_G_slices(int N, double L, int K, const double *radii, int m,
                      const or_atten *at, int conserve, double *G)
{
    const int64_t n3 = (int64_t)N * N * N;
    memset(G, 0, sizeof(double) * n3 * K);
    for (int k = 0; k < K; ++k) {
        kern_t kp;
        if (kern_init(&kp, N, L, K, radii, m, &at[k])) return -1;
        double *Gk = G + (int64_t)k * n3;
        #pragma omp parallel for schedule(dynamic, 64)
        for (int64_t c = 0; c < n3; ++c) {
            int i = (int)(c / ((int64_t)N * N)), j = (int)((c / N) % N), x = (int)(c % N);
            double v = 0.0;
            kern_accumulate(&kp, i, j, x, k, k + 1, &v);
            Gk[c] = v;
        }
        if (conserve) {
            double l3 = kp.l * kp.l * kp.l, s = 0.0, comp = 0.0;
            for (int64_t c = 0; c < n3; ++c) {
                double v = Gk[c], t = s + v;
                comp += (fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s;
                s = t;
            }
            s += comp;
            double target = or_shell_integral(&at[k], radii[k], radii[k + 1]);
            double f = (s != 0.0) ? target / (l3 * s) : 0.0;
            for (int64_t c = 0; c < n3; ++c) Gk[c] *= f;
        }
    }
    return 0;
}

/* ---- near-field (particle-mesh) correction (Sec. 4) -------------------
 * Sources with positions x_s inside their cells sit on their nearest node
 * c_s = round(x_s / l) in the mesh field. For target nodes c_s + o with
 * 0 < max|o_d| <= R the primary-image part of the mesh kernel, the
 * m^3-subpoint average over the image u = 0 at displacement o, is replaced
 * by the retarded kernel at the exact distance |(c_s + o) l - x_s|
 * (with rule 1, the primary image's exact cell average is replaced):
 *   corr(c_s + o) += L (F_k(rho) - Gprim_k(o)).
 * Slice k of the K point lists uses at[k]. Plain sequential FP64 sums. */
static double or_G_primary(const kern_t *kp, int k, int o0, int o1, int o2)
{
    const int m = kp->m;
    double acc = 0.0;
    for (int a0 = 0; a0 < m; ++a0)
    for (int a1 = 0; a1 < m; ++a1)
    for (int a2 = 0; a2 < m; ++a2) {
        int64_t q0 = 2 * m * (int64_t)o0 + (2 * a0 + 1 - m);
        int64_t q1 = 2 * m * (int64_t)o1 + (2 * a1 + 1 - m);
        int64_t q2 = 2 * m * (int64_t)o2 + (2 * a2 + 1 - m);
        int64_t n = q0 * q0 + q1 * q1 + q2 * q2;
        double dn = (double)n;
        if (dn >= kp->T[k] && dn < kp->T[k + 1]) acc += point_value(kp, n);
    }
    return acc;
}

double or_cell_average(const or_atten *at, double l, const double *B, double rlo, double rhi, int ng);

/* rule 1: the mesh kernel is the exact cell average (or_cell_average of the
 * primary image cell) instead of the subpoint average */
int or_near_correction(int N, double L, int K, const double *radii, int m, const or_atten *at,
                       const int64_t *off, const double *pos, const double *lum, int R, double *corr,
                       int rule, int ng)
{
    const double l = L / N;
    const int D = 2 * R + 1;
    memset(corr, 0, sizeof(double) * (int64_t)N * N * N);
    double *Gtab = (double *)malloc(sizeof(double) * D * D * D);
    if (!Gtab) return -1;
    for (int k = 0; k < K; ++k) {
        kern_t kp;
        if (kern_init(&kp, N, L, K, radii, m, &at[k])) { free(Gtab); return -1; }
        /* the primary image's mesh kernel at every offset of slice k (it
         * depends on the offset only) */
        #pragma omp parallel for schedule(dynamic, 1)
        for (int t = 0; t < D * D * D; ++t) {
            int o0 = t / (D * D) - R, o1 = (t / D) % D - R, o2 = t % D - R;
            if (rule == 1) {
                double B[6] = { (o0 - 0.5) * l, (o0 + 0.5) * l, (o1 - 0.5) * l, (o1 + 0.5) * l,
                                (o2 - 0.5) * l, (o2 + 0.5) * l };
                Gtab[t] = or_cell_average(&at[k], l, B, radii[k], radii[k + 1], ng);
            } else {
                Gtab[t] = or_G_primary(&kp, k, o0, o1, o2);
            }
        }
        for (int64_t s = off[k]; s < off[k + 1]; ++s) {
            double c[3];
            for (int d = 0; d < 3; ++d) c[d] = floor(pos[3 * s + d] / l + 0.5);
            for (int o0 = -R; o0 <= R; ++o0)
            for (int o1 = -R; o1 <= R; ++o1)
            for (int o2 = -R; o2 <= R; ++o2) {
                if (o0 == 0 && o1 == 0 && o2 == 0) continue;
                int o[3] = { o0, o1, o2 };
                double r2 = 0.0;
                int64_t cell = 0;
                for (int d = 0; d < 3; ++d) {
                    double y = (c[d] + o[d]) * l - pos[3 * s + d];
                    r2 += y * y;
                    int64_t v = ((int64_t)c[d] + o[d]) % N;
                    if (v < 0) v += N;
                    cell = cell * N + v;
                }
                double rho = sqrt(r2);
                double F = 0.0;
                if (rho >= radii[k] && rho < radii[k + 1])
                    F = at[k].prefactor * or_phi(&at[k], rho) / (4.0 * OR_PI * rho * rho);
                double Gp = Gtab[((o0 + R) * D + (o1 + R)) * D + (o2 + R)];
                corr[cell] += lum[s] * (F - Gp);
            }
        }
    }
    free(Gtab);
    return 0;
}

/* ---- exact cell-averaged kernel ----------------------------------------
 * The m -> infinity limit of the subpoint average (the "exact cell
 * integral" refinement of the near-source treatment of Sec. 4). For an image
 * cell B = [x0,x1] x [y0,y1] x [z0,z1] of the unit source at the origin and
 * the shell [r_lo, r_hi) of Eq. 10:
 *
 *   G_B = pref / l^3 * int_B phi(|x|) / (4 pi |x|^2) [r_lo <= |x| < r_hi] d^3x.
 *
 * Cylindrical coordinates about the z axis (x = R cos t, y = R sin t,
 * d^3x = R dR dt dz) and z = R tan s (so |x| = R / cos s and
 * dz / |x|^2 = ds / R) turn it into
 *
 *   G_B = pref / (4 pi l^3) int_R Theta(R) S(R) dR,
 *   Theta(R) = angle of the circle of radius R inside [x0,x1] x [y0,y1],
 *   S(R)     = int_{A(R)} phi(R / cos s) ds,
 *   A(R)     = {s in (-pi/2, pi/2): z0 <= R tan s <= z1, r_lo <= R / cos s < r_hi}.
 *
 * With phi = 1, S(R) is the length of A(R) and G_B is a single quadrature
 * in R. R is split wherever Theta or A(R) changes form (edge and corner
 * distances of the rectangle, r_lo, r_hi, sqrt(r^2 - z^2) for the z faces);
 * each piece is integrated by ng-point Gauss-Legendre after the substitution
 * R = Ra + (Rb - Ra)(1 - cos u)/2, u in [0, pi], which turns the square-root
 * behaviour at the piece ends into smooth integrands, bisected until the
 * halves agree with the whole. A piece starting at
 * R = 0 (cells around the source) takes the tanh-sinh rule instead: there
 * S(R) carries the r^p cusp of phi at r = 0 (S(R) ~ S(0) - C R^p), an
 * algebraic end singularity that the substitution does not remove. The phi
 * integral over
 * each interval of A(R) (kinds 1 and 2, whose support ends are folded into
 * r_hi) is an ng-point Gauss-Legendre rule. */

/* angle of the circle of radius R inside [a,b] x [c,d], 0 <= a < b, 0 <= c < d
 * (first quadrant): x = R cos t in [a,b] and y = R sin t in [c,d] */
static double theta_quadrant(double R, double a, double b, double c, double d)
{
    double tx0 = acos(fmin(1.0, a / R)), tx1 = acos(fmin(1.0, b / R));
    double ty0 = asin(fmin(1.0, c / R)), ty1 = asin(fmin(1.0, d / R));
    double lo = fmax(tx1, ty0), hi = fmin(tx0, ty1);
    return hi > lo ? hi - lo : 0.0;
}

/* Theta(R): the rectangle's parts in the four quadrants, each reflected into
 * the first one. */
double or_theta_rect(double R, double x0, double x1, double y0, double y1)
{
    if (!(R > 0.0)) return 0.0;
    double t = 0.0;
    for (int sx = 0; sx < 2; ++sx)
    for (int sy = 0; sy < 2; ++sy) {
        double a = sx == 0 ? fmax(x0, 0.0) : fmax(-x1, 0.0);
        double b = sx == 0 ? x1 : -x0;
        double c = sy == 0 ? fmax(y0, 0.0) : fmax(-y1, 0.0);
        double d = sy == 0 ? y1 : -y0;
        if (b > a && d > c) t += theta_quadrant(R, a, b, c, d);
    }
    return t;
}

/* S(R) for R > 0; rhi is already capped at the end of phi's support */
static double s_of_R(const or_atten *at, double R, double z0, double z1, double rlo, double rhi,
                     int ng, const double *gx, const double *gw)
{
    if (R >= rhi) return 0.0;
    double tH = acos(R / rhi);
    double tL = R < rlo ? acos(R / rlo) : 0.0;
    double ta = atan2(z0, R), tb = atan2(z1, R);
    double iv[2][2] = { { fmax(ta, -tH), fmin(tb, -tL) }, { fmax(ta, tL), fmin(tb, tH) } };
    double acc = 0.0;
    for (int i = 0; i < 2; ++i) {
        double lo = iv[i][0], hi = iv[i][1];
        if (!(hi > lo)) continue;
        if (at->kind == 0) { acc += hi - lo; continue; }
        /* tanh-sinh in s: for small R, phi(R / cos s) changes within thin
         * layers at the interval ends (|s| near pi/2), which the rule's
         * end clustering resolves. s = mid + hw tanh(y), y = (pi/2) sinh t;
         * the distance to the nearer end, hw / (1 + e^{2|y|}), is formed
         * directly so that cos s keeps its relative accuracy there. */
        double hw = 0.5 * (hi - lo), mid = 0.5 * (hi + lo), q = 0.0;
        const double h = 2.0 / ng;
        const int nt = (int)(4.0 / h);
        for (int j = -nt; j <= nt; ++j) {
            double t = j * h, y = 0.5 * OR_PI * sinh(t);
            double dist = 2.0 * hw / (1.0 + exp(2.0 * fabs(y)));   /* to the end on y's side */
            double sv = y >= 0.0 ? hi - dist : lo + dist;
            double cy = cosh(y);
            double w = h * hw * 0.5 * OR_PI * cosh(t) / (cy * cy);
            if (!(w > 0.0)) continue;
            q += w * or_phi(at, R / cos(sv));
        }
        acc += q;
    }
    return acc;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct {
    const or_atten *at;
    double x0, x1, y0, y1, z0, z1, rlo, rhi;
    int ng;
    const double *gx, *gw;
} cell_ctx;

/* ng-point Gauss-Legendre rule for int_a^b Theta(R) S(R) dR after
 * R = a + (b - a)(1 - cos u)/2 */
static double piece_gl(const cell_ctx *c, double a, double b)
{
    double q = 0.0;
    for (int j = 0; j < c->ng; ++j) {
        double u = 0.5 * OR_PI * (c->gx[j] + 1.0);
        double R = a + 0.5 * (b - a) * (1.0 - cos(u));
        double jac = 0.5 * OR_PI * 0.5 * (b - a) * sin(u);
        q += c->gw[j] * jac * or_theta_rect(R, c->x0, c->x1, c->y0, c->y1) *
             s_of_R(c->at, R, c->z0, c->z1, c->rlo, c->rhi, c->ng, c->gx, c->gw);
    }
    return q;
}

/* Adaptive bisection: the two halves replace the whole until they agree
 * with it to tol (absolute: a small multiple of the rounding level of the
 * whole cell's value), after at least two levels (an early agreement of
 * two poor estimates is not taken). A piece is analytic inside, but a
 * breakpoint just outside it (a shell radius close to an edge distance,
 * say) slows the rule's convergence; halving towards it restores it. */
static double piece_adapt(const cell_ctx *c, double a, double b, double whole, double tol, int depth,
                          int *budget)
{
    double m = 0.5 * (a + b);
    double lq = piece_gl(c, a, m), rq = piece_gl(c, m, b);
    double two = lq + rq;
    if (depth >= 48 || *budget <= 0 || (depth >= 2 && fabs(two - whole) <= tol)) return two;
    *budget -= 2;
    return piece_adapt(c, a, m, lq, 0.5 * tol, depth + 1, budget) +
           piece_adapt(c, m, b, rq, 0.5 * tol, depth + 1, budget);
}

/* G_B for the box B = {x0,x1,y0,y1,z0,z1} (length units, source at the
 * origin), shell [rlo, rhi), cell side l, ng-point rules (ng <= 64). */
double or_cell_average(const or_atten *at, double l, const double *B, double rlo, double rhi, int ng)
{
    if (ng < 2 || ng > 64) return NAN;
    double sup = phi_support_end(at);
    if (rhi > sup) rhi = sup;
    if (!(rhi > rlo)) return 0.0;
    const double x0 = B[0], x1 = B[1], y0 = B[2], y1 = B[3], z0 = B[4], z1 = B[5];
    double nx = x0 > 0.0 ? x0 : (x1 < 0.0 ? -x1 : 0.0);
    double ny = y0 > 0.0 ? y0 : (y1 < 0.0 ? -y1 : 0.0);
    double Rmin = hypot(nx, ny);
    double Rmax = fmin(hypot(fmax(fabs(x0), fabs(x1)), fmax(fabs(y0), fabs(y1))), rhi);
    if (!(Rmax > Rmin)) return 0.0;
    double br[32];
    int nb = 0;
    br[nb++] = Rmin;
    br[nb++] = Rmax;
    const double xs[2] = { x0, x1 }, ys[2] = { y0, y1 }, zs[2] = { z0, z1 }, rs[2] = { rlo, rhi };
    double cand[16];
    int nc = 0;
    for (int i = 0; i < 2; ++i) { cand[nc++] = fabs(xs[i]); cand[nc++] = fabs(ys[i]); }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) cand[nc++] = hypot(xs[i], ys[j]);
    cand[nc++] = rlo;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (rs[i] > fabs(zs[j])) cand[nc++] = sqrt(rs[i] * rs[i] - zs[j] * zs[j]);
    for (int i = 0; i < nc; ++i)
        if (cand[i] > Rmin && cand[i] < Rmax) br[nb++] = cand[i];
    qsort(br, nb, sizeof(double), cmp_double);
    double gx[64], gw[64];
    gauss_legendre(ng, gx, gw);
    cell_ctx cc = { at, x0, x1, y0, y1, z0, z1, rlo, rhi, ng, gx, gw };
    /* scale of the whole cell's value (plain rule on every piece) */
    double est = 0.0;
    for (int p = 0; p + 1 < nb; ++p)
        if (br[p + 1] > br[p]) est += fabs(piece_gl(&cc, br[p], br[p + 1]));
    const double tol = 1e-14 * est;
    double acc = 0.0;
    for (int p = 0; p + 1 < nb; ++p) {
        double Ra = br[p], Rb = br[p + 1];
        if (!(Rb > Ra)) continue;
        double q = 0.0;
        if (Ra == 0.0) {
            /* tanh-sinh: R = Rb / (1 + e^{-2y}), y = (pi/2) sinh t, t in
             * [-4, 4] with step 1/(ng/2); dR/dt = Rb (pi/2) cosh t /
             * (2 cosh^2 y) */
            const double h = 2.0 / ng;
            const int nt = (int)(4.0 / h);
            for (int i = -nt; i <= nt; ++i) {
                double t = i * h, y = 0.5 * OR_PI * sinh(t);
                double R = Rb / (1.0 + exp(-2.0 * y));
                double cy = cosh(y);
                double w = h * Rb * 0.5 * OR_PI * cosh(t) / (2.0 * cy * cy);
                if (!(R > 0.0) || !(w > 0.0)) continue;
                q += w * or_theta_rect(R, x0, x1, y0, y1) * s_of_R(at, R, z0, z1, rlo, rhi, ng, gx, gw);
            }
            acc += q;
            continue;
        }
        int budget = 512;
        acc += piece_adapt(&cc, Ra, Rb, piece_gl(&cc, Ra, Rb), tol, 0, &budget);
    }
    return at->prefactor * acc / (4.0 * OR_PI * l * l * l);
}

/* All K exact shell values at displacement (d0,d1,d2) (cells), every
 * periodic image whose cell can reach [r_0, r_K) (the culling of
 * kern_accumulate). */
static void exact_accumulate(int N, double L, int K, const double *radii, const or_atten *at,
                             int d0, int d1, int d2, int ng, double *outK)
{
    const double l = L / N;
    const int U = (int)ceil(radii[K] / L) + 1;
    int dd[3] = { ((d0 % N) + N) % N, ((d1 % N) + N) % N, ((d2 % N) + N) % N };
    for (int u0 = -U; u0 <= U; ++u0)
    for (int u1 = -U; u1 <= U; ++u1)
    for (int u2 = -U; u2 <= U; ++u2) {
        int64_t cx[3] = { dd[0] + (int64_t)u0 * N, dd[1] + (int64_t)u1 * N, dd[2] + (int64_t)u2 * N };
        double B[6], mn2 = 0.0, mx2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double lo = ((double)cx[a] - 0.5) * l, hi = ((double)cx[a] + 0.5) * l;
            B[2 * a] = lo; B[2 * a + 1] = hi;
            double near = lo > 0.0 ? lo : (hi < 0.0 ? -hi : 0.0), far = fmax(fabs(lo), fabs(hi));
            mn2 += near * near; mx2 += far * far;
        }
        if (sqrt(mn2) >= radii[K] || sqrt(mx2) <= radii[0]) continue;
        for (int k = 0; k < K; ++k) {
            if (sqrt(mn2) >= radii[k + 1] || sqrt(mx2) <= radii[k]) continue;
            outK[k] += or_cell_average(at, l, B, radii[k], radii[k + 1], ng);
        }
    }
}

int or_G_exact_at(int N, double L, int K, const double *radii, const or_atten *at,
                  int d0, int d1, int d2, int ng, double *outK)
{
    if (K < 1 || ng < 2 || ng > 64) return -1;
    memset(outK, 0, sizeof(double) * K);
    exact_accumulate(N, L, K, radii, at, d0, d1, d2, ng, outK);
    return 0;
}

/* Dense exact kernel G[k][i][j][kx] (no rescaling: the exact cell average
 * already sums to the shell integral over the cells reached). */
int or_build_G_exact(int N, double L, int K, const double *radii, const or_atten *at, int ng, double *G)
{
    if (K < 1 || ng < 2 || ng > 64) return -1;
    const int64_t n3 = (int64_t)N * N * N;
    memset(G, 0, sizeof(double) * n3 * K);
    #pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * K);
        #pragma omp for schedule(dynamic, 16)
        for (int64_t c = 0; c < n3; ++c) {
            int i = (int)(c / ((int64_t)N * N)), j = (int)((c / N) % N), x = (int)(c % N);
            memset(tmp, 0, sizeof(double) * K);
            exact_accumulate(N, L, K, radii, at, i, j, x, ng, tmp);
            for (int k = 0; k < K; ++k) G[(int64_t)k * n3 + c] = tmp[k];
        }
        free(tmp);
    }
    return 0;
}

/* ---- naive DFT (Eq. 12 convention) ------------------------------------- */

/* Twiddle table e^{sign 2 pi i j / N}, j in [0, N), from long double libm. */
static void twiddles(int N, int sign, double complex *w)
{
    for (int j = 0; j < N; ++j) {
        long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)j / (long double)N;
        w[j] = (double)cosl(ang) + (double)(sign * sinl(ang)) * I;
    }
}

/* In-place separable naive DFT of a complex N^3 array along all three axes.
 * sign = -1: forward (unnormalised); +1: inverse (unnormalised). */
int or_dft3_naive(int N, int sign, double complex *a)
{
    double complex *w = (double complex *)malloc(sizeof(double complex) * N);
    twiddles(N, sign, w);
    const int64_t NN = (int64_t)N * N;
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t st = (ax == 0) ? NN : (ax == 1) ? N : 1;
        #pragma omp parallel
        {
            double complex *line = (double complex *)malloc(sizeof(double complex) * N);
            #pragma omp for schedule(static)
            for (int64_t ln = 0; ln < NN; ++ln) {
                /* the two coordinates other than ax */
                int64_t hi = ln / N, lo = ln % N;
                int64_t base = (ax == 0) ? hi * N + lo
                             : (ax == 1) ? hi * NN + lo
                                         : (hi * N + lo) * N;
                for (int j = 0; j < N; ++j) line[j] = a[base + j * st];
                for (int p = 0; p < N; ++p) {
                    double complex acc = 0.0;
                    for (int j = 0; j < N; ++j)
                        acc += line[j] * w[((int64_t)j * p) % N];
                    a[base + p * st] = acc;
                }
            }
            free(line);
        }
    }
    free(w);
    return 0;
}

/* Brute-force non-separable 3D DFT, O(N^6). */
int or_dft3_brute(int N, int sign, const double complex *in, double complex *out)
{
    double complex *w = (double complex *)malloc(sizeof(double complex) * N);
    twiddles(N, sign, w);
    const int64_t n3 = (int64_t)N * N * N;
    #pragma omp parallel for schedule(static)
    for (int64_t P = 0; P < n3; ++P) {
        int p = (int)(P / ((int64_t)N * N)), q = (int)((P / N) % N), r = (int)(P % N);
        double complex acc = 0.0;
        for (int64_t c = 0; c < n3; ++c) {
            int i = (int)(c / ((int64_t)N * N)), j = (int)((c / N) % N), k = (int)(c % N);
            acc += in[c] * w[((int64_t)i * p + (int64_t)j * q + (int64_t)k * r) % N];
        }
        out[P] = acc;
    }
    free(w);
    return 0;
}

/* Brute-force circular convolution, O(N^6): out(x) = sum_c G((x-c) mod N) S(c). */
int or_conv3_brute(int N, const double *G, const double *S, double *out)
{
    const int64_t n3 = (int64_t)N * N * N;
    #pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < n3; ++x) {
        int xi = (int)(x / ((int64_t)N * N)), xj = (int)((x / N) % N), xk = (int)(x % N);
        nsum acc = { 0.0, 0.0 };
        for (int64_t c = 0; c < n3; ++c) {
            if (S[c] == 0.0) continue;
            int ci = (int)(c / ((int64_t)N * N)), cj = (int)((c / N) % N), ck = (int)(c % N);
            int64_t d = ((int64_t)((xi - ci + N) % N) * N + (xj - cj + N) % N) * N + (xk - ck + N) % N;
            nadd(&acc, G[d] * S[c]);
        }
        out[x] = acc.s + acc.c;
    }
    return 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

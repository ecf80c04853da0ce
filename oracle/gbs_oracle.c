/*
 * Plain FP64 reference ("oracle") for Gaussian beam summation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the HIP library is checked against.  It shares no code,
 * header, table or constant with the library; only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.
 *
 * What it computes (paper Sec. 2):
 *
 *   Eq. (1) gives the field of one Gaussian beam in ray-centred coordinates,
 *   amplitude sqrt(det Q0 / det Q) and exponent
 *   i*omega*(tau + 1/2 q^T (P Q^-1) q).  We take the isotropic 3-D beam
 *   P = p I, Q = q I, so det Q0 / det Q = (q0/q)^2 and the amplitude is q0/q.
 *
 *   Eq. (2) (dQ/ds = c P, dP/ds = 0) in a homogeneous medium gives p = 1/c
 *   constant and q(s) = q0 + s with q0 = -i*eps (eps > 0: the beam decays away
 *   from its axis under the exp(-i omega t) convention of Eq. (1)).
 *
 *   Eq. (3) sums beams over the launch parameters with a weighting function.
 *   Discretised over rays j with launch solid angle w_j, the weight per ray is
 *   (i k / 2 pi) w_j / (4 pi): the stationary-phase value of the beam integral
 *   that reproduces a unit monopole exp(i k r) / (4 pi r) in free field.
 *   A reflected beam carries the product of the reflection coefficients of
 *   the faces it has hit (angle independent).
 *
 * For receiver R and segment j (start a, unit axis t, arc length s0 at a,
 * beam interval [lo, hi) in sigma):
 *
 *   sigma = (R - a).t        keep iff lo <= sigma < hi
 *   n^2   = |R - a|^2 - sigma^2            (squared normal distance)
 *   s     = s0 + sigma,  q = q0 + s,  tau = s / c
 *   E     = i omega (tau + 1/2 (p/q) n^2)  keep iff Re E >= -G
 *   u     = (i k w_j / (8 pi^2)) * prod Gamma * (q0 / q) * exp(E)
 *   P(R)  = sum_j u,   TL = -20 log10 |P|
 *
 * Atmospheric absorption (optional, per job): the pressure amplitude of a
 * beam decays as exp(-alpha s) along its arc length, alpha in Np/m (the
 * paper's atmosphere of Tables 2 and 3: temperature, humidity, pressure;
 * alpha from the pure-tone attenuation of ISO 9613-1, gbso_air_absorption_db).
 *
 * Sums are Neumaier-compensated, in table order.  Jobs are (source, band)
 * pairs, job = src * n_freq + band; eps is given per job.  Optionally the
 * sum of |u| is returned: |P| / sum |u| measures the cancellation in the sum
 * (near interference nulls it is small and TL is ill-conditioned).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define PI 3.14159265358979323846

/* Neumaier (improved Kahan) running sum of doubles. */
typedef struct { double sum, comp; } nsum;

static void nsum_add(nsum* a, double x) {
    double t = a->sum + x;
    if (fabs(a->sum) >= fabs(x))
        a->comp += (a->sum - t) + x;
    else
        a->comp += (x - t) + a->sum;
    a->sum = t;
}

static double nsum_get(const nsum* a) { return a->sum + a->comp; }

/* Product of the reflection coefficients of the faces a segment has hit. */
static cplx face_product(const int64_t* face_ptr, const int32_t* face_ids, const double* gamma, int64_t j) {
    cplx g = 1.0;
    for (int64_t m = face_ptr[j]; m < face_ptr[j + 1]; ++m) {
        int32_t f = face_ids[m];
        g *= gamma[2 * f] + I * gamma[2 * f + 1];
    }
    return g;
}

/* Derivative of the face product with respect to Gamma_f (holomorphic):
 * sum over the occurrences of f of the product of the other factors. */
static cplx face_product_deriv(const int64_t* face_ptr, const int32_t* face_ids, const double* gamma,
                               int64_t j, int32_t f) {
    cplx d = 0.0;
    for (int64_t l = face_ptr[j]; l < face_ptr[j + 1]; ++l) {
        if (face_ids[l] != f) continue;
        cplx others = 1.0;
        for (int64_t m = face_ptr[j]; m < face_ptr[j + 1]; ++m) {
            if (m == l) continue;
            int32_t g = face_ids[m];
            others *= gamma[2 * g] + I * gamma[2 * g + 1];
        }
        d += others;
    }
    return d;
}

/* Geometry of one (receiver, segment) pair; returns whether sigma lies in
 * the segment's beam interval [lo, hi). */
typedef struct {
    double sigma, n2, s;
    double v[3];      /* R - a */
} pair_geom;

static int pair_geometry(const double* R, const double* a, const double* t, double s0, double lo, double hi,
                         pair_geom* g) {
    g->v[0] = R[0] - a[0];
    g->v[1] = R[1] - a[1];
    g->v[2] = R[2] - a[2];
    g->sigma = g->v[0] * t[0] + g->v[1] * t[1] + g->v[2] * t[2];
    double vv = g->v[0] * g->v[0] + g->v[1] * g->v[1] + g->v[2] * g->v[2];
    g->n2 = vv - g->sigma * g->sigma;
    if (g->n2 < 0.0) g->n2 = 0.0;
    g->s = s0 + g->sigma;
    return lo <= g->sigma && g->sigma < hi;
}

/* Beam exponent E = i omega (tau + 1/2 (p/q) n^2) and q for a pair. */
static cplx beam_exponent(double omega, double c, double eps, double s, double n2, cplx* q_out) {
    cplx q0 = -I * eps;
    cplx q = q0 + s;
    double p = 1.0 / c;
    double tau = s / c;
    *q_out = q;
    return I * omega * (tau + 0.5 * (p / q) * n2);
}

/* mask_mode: 0 gate normally; 1 gate normally and record the active set in
 * mask[job][rcv][seg]; 2 use the recorded active set instead of the gate
 * (frozen-mask evaluation for finite differences). */
int gbso_forward(int32_t n_src, int64_t n_rays, const int64_t* ray_ptr, const double* ray_w,
                 const int32_t* ray_src, int64_t n_segs, const double* seg_a, const double* seg_t,
                 const double* seg_s0, const double* seg_lo, const double* seg_hi, const int64_t* face_ptr,
                 const int32_t* face_ids, int32_t n_faces, const double* gamma, int64_t n_rcv,
                 const double* rcv, int32_t n_freq, const double* freqs, const double* eps,
                 const double* alpha, double c, double gate_G, int32_t n_threads, int32_t mask_mode,
                 uint8_t* mask, double* P_out,
                 double* TL_out, double* absum_out) {
    (void)n_faces;
    if (n_src < 0 || n_rays < 0 || n_segs < 0 || n_rcv < 0 || n_freq < 0 || c <= 0) return -1;
    if (mask_mode != 0 && mask == NULL) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    for (int32_t src = 0; src < n_src; ++src) {
        for (int32_t b = 0; b < n_freq; ++b) {
            const int64_t job = (int64_t)src * n_freq + b;
            const double omega = 2.0 * PI * freqs[b];
            const double k = omega / c;
            const double e = eps[job];
            const double al = alpha ? alpha[job] : 0.0;
#pragma omp parallel for schedule(dynamic, 16) if (n_threads != 1)
            for (int64_t r = 0; r < n_rcv; ++r) {
                const double* R = rcv + 3 * r;
                nsum re = {0, 0}, im = {0, 0}, ab = {0, 0};
                for (int64_t i = 0; i < n_rays; ++i) {
                    if (ray_src[i] != src) continue;
                    const cplx weight = I * k * ray_w[i] / (8.0 * PI * PI);
                    for (int64_t j = ray_ptr[i]; j < ray_ptr[i + 1]; ++j) {
                        pair_geom g;
                        int inside = pair_geometry(R, seg_a + 3 * j, seg_t + 3 * j, seg_s0[j], seg_lo[j],
                                                   seg_hi[j], &g);
                        cplx q;
                        cplx E = beam_exponent(omega, c, e, g.s, g.n2, &q);
                        int active = inside && creal(E) >= -gate_G;
                        if (mask_mode == 1) mask[(job * n_rcv + r) * n_segs + j] = (uint8_t)active;
                        if (mask_mode == 2) active = mask[(job * n_rcv + r) * n_segs + j];
                        if (!active) continue;
                        cplx q0 = -I * e;
                        cplx u = weight * face_product(face_ptr, face_ids, gamma, j) * (q0 / q) * cexp(E) *
                                 exp(-al * g.s);
                        nsum_add(&re, creal(u));
                        nsum_add(&im, cimag(u));
                        nsum_add(&ab, cabs(u));
                    }
                }
                double pr = nsum_get(&re), pi = nsum_get(&im);
                if (absum_out) absum_out[job * n_rcv + r] = nsum_get(&ab);
                P_out[2 * (job * n_rcv + r)] = pr;
                P_out[2 * (job * n_rcv + r) + 1] = pi;
                double mag = hypot(pr, pi);
                TL_out[job * n_rcv + r] = mag > 0 ? -20.0 * log10(mag) : INFINITY;
            }
        }
    }
    return 0;
}

/*
 * Anisotropic beams: Eq. (1) with a 2x2 Q.  Ray-centred coordinates (s, q1, q2)
 * measure the normal offset along unit vectors e1 and e2 = t x e1 (both normal
 * to the axis t).  Eq. (2) in a homogeneous medium with P = I / c and the
 * initial Q0 = diag(-i eps1, -i eps2) gives Q(s) = diag(q1, q2) with
 * q_m = s - i eps_m, hence
 *
 *   amplitude  sqrt(det Q0 / det Q) = sqrt(q01 / q1) * sqrt(q02 / q2)
 *   exponent   E = i omega (tau + 1/2 p (n1^2 / q1 + n2^2 / q2)),
 *              n_m = (R - a).e_m        keep iff Re E >= -G
 *
 * Each ratio q0m / qm = eps_m (eps_m - i s) / |q_m|^2 has a positive real part
 * for every real s, so the principal square root is the branch that is
 * continuous along the beam (and equals 1 at s = 0): no branch tracking is
 * needed.  A planar reflection maps the frame by the mirror, which leaves n1^2
 * and n2^2 unchanged, so the frame of a reflected segment is the mirror image
 * of the incident one (the sign of e1 does not matter).  eps1 = eps[job] is the
 * beam parameter along e1, eps2 = eps_e2[job] along e2; with eps1 = eps2 the
 * beam is the isotropic one of gbso_forward.  seg_e1[3 j..] is e1 of segment j.
 */
/* Ray-centred coordinates of a pair for anisotropic beams: the offsets n1, n2
 * of R along e1 and e2 = t x e1 (v = R - a from pair_geometry). */
static void frame_offsets(const pair_geom* g, const double* t, const double* f1, double* n1, double* n2,
                          double f2[3]) {
    f2[0] = t[1] * f1[2] - t[2] * f1[1];
    f2[1] = t[2] * f1[0] - t[0] * f1[2];
    f2[2] = t[0] * f1[1] - t[1] * f1[0];
    *n1 = g->v[0] * f1[0] + g->v[1] * f1[1] + g->v[2] * f1[2];
    *n2 = g->v[0] * f2[0] + g->v[1] * f2[1] + g->v[2] * f2[2];
}

/* mask_mode as for gbso_forward (0: gate; 1: gate and record; 2: recorded set). */
int gbso_forward_aniso(int32_t n_src, int64_t n_rays, const int64_t* ray_ptr, const double* ray_w,
                       const int32_t* ray_src, int64_t n_segs, const double* seg_a, const double* seg_t,
                       const double* seg_s0, const double* seg_lo, const double* seg_hi, const int64_t* face_ptr,
                       const int32_t* face_ids, int32_t n_faces, const double* gamma, int64_t n_rcv,
                       const double* rcv, int32_t n_freq, const double* freqs, const double* eps,
                       const double* alpha, double c, double gate_G, const double* eps_e2, const double* seg_e1,
                       int32_t n_threads, int32_t mask_mode, uint8_t* mask, double* P_out, double* TL_out,
                       double* absum_out) {
    (void)n_faces;
    if (n_src < 0 || n_rays < 0 || n_segs < 0 || n_rcv < 0 || n_freq < 0 || c <= 0) return -1;
    if (eps_e2 == NULL || (n_segs > 0 && seg_e1 == NULL)) return -1;
    if (mask_mode != 0 && mask == NULL) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    for (int32_t src = 0; src < n_src; ++src) {
        for (int32_t b = 0; b < n_freq; ++b) {
            const int64_t job = (int64_t)src * n_freq + b;
            const double omega = 2.0 * PI * freqs[b];
            const double k = omega / c;
            const double p = 1.0 / c;
            const double e1 = eps[job], e2 = eps_e2[job];
            const double al = alpha ? alpha[job] : 0.0;
#pragma omp parallel for schedule(dynamic, 16) if (n_threads != 1)
            for (int64_t r = 0; r < n_rcv; ++r) {
                const double* R = rcv + 3 * r;
                nsum re = {0, 0}, im = {0, 0}, ab = {0, 0};
                for (int64_t i = 0; i < n_rays; ++i) {
                    if (ray_src[i] != src) continue;
                    const cplx weight = I * k * ray_w[i] / (8.0 * PI * PI);
                    for (int64_t j = ray_ptr[i]; j < ray_ptr[i + 1]; ++j) {
                        pair_geom g;
                        const double* t = seg_t + 3 * j;
                        const int inside = pair_geometry(R, seg_a + 3 * j, t, seg_s0[j], seg_lo[j], seg_hi[j], &g);
                        double n1, n2, f2[3];
                        frame_offsets(&g, t, seg_e1 + 3 * j, &n1, &n2, f2);
                        const cplx q01 = -I * e1, q02 = -I * e2;
                        const cplx q1 = q01 + g.s, q2 = q02 + g.s;
                        const cplx E = I * omega * (g.s / c + 0.5 * p * (n1 * n1 / q1 + n2 * n2 / q2));
                        int active = inside && creal(E) >= -gate_G;
                        if (mask_mode == 1) mask[(job * n_rcv + r) * n_segs + j] = (uint8_t)active;
                        if (mask_mode == 2) active = mask[(job * n_rcv + r) * n_segs + j];
                        if (!active) continue;
                        const cplx amp = csqrt(q01 / q1) * csqrt(q02 / q2);
                        const cplx u = weight * face_product(face_ptr, face_ids, gamma, j) * amp * cexp(E) *
                                       exp(-al * g.s);
                        nsum_add(&re, creal(u));
                        nsum_add(&im, cimag(u));
                        nsum_add(&ab, cabs(u));
                    }
                }
                double pr = nsum_get(&re), pi = nsum_get(&im);
                if (absum_out) absum_out[job * n_rcv + r] = nsum_get(&ab);
                P_out[2 * (job * n_rcv + r)] = pr;
                P_out[2 * (job * n_rcv + r) + 1] = pi;
                double mag = hypot(pr, pi);
                TL_out[job * n_rcv + r] = mag > 0 ? -20.0 * log10(mag) : INFINITY;
            }
        }
    }
    return 0;
}

/*
 * Hand-derived adjoint.  With dL = Re sum_{job,r} lambda[job,r] dP[job,r]:
 *
 *   d ln u / dR   = t (ik - 1/q - (ik/2) n^2 / q^2 - alpha) + (ik/q) nvec,
 *                   nvec = (R - a) - sigma t   (dq/dR = t, d(n^2)/dR = 2 nvec)
 *   d ln u / deps = 1/eps + i/q - (k/2) n^2 / q^2
 *                   (weight*q0 is proportional to eps; dq/deps = -i)
 *   dP / dGamma_f = sum_j (d prod Gamma_j / dGamma_f) * u_j / prod Gamma_j
 *                   computed without dividing: u_j / prod Gamma_j is the
 *                   beam term with the coefficient product left out.
 *
 * Outputs: d_rcv[r][3] = Re(sum_job lambda * sum_j u * dln u/dR);
 *          d_eps[job]  = Re(sum_r lambda * sum_j u * dln u/deps);
 *          d_gamma[f]  = (Re Z_f, -Im Z_f) = (dL/dRe Gamma_f, dL/dIm Gamma_f),
 *          Z_f = sum_{job,r} lambda * dP/dGamma_f.
 * The gate is taken as fixed (almost-everywhere derivative); mask_mode 2
 * uses a recorded active set.
 */
int gbso_backward(int32_t n_src, int64_t n_rays, const int64_t* ray_ptr, const double* ray_w,
                  const int32_t* ray_src, int64_t n_segs, const double* seg_a, const double* seg_t,
                  const double* seg_s0, const double* seg_lo, const double* seg_hi, const int64_t* face_ptr,
                  const int32_t* face_ids, int32_t n_faces, const double* gamma, int64_t n_rcv,
                  const double* rcv, int32_t n_freq, const double* freqs, const double* eps,
                  const double* alpha, double c, double gate_G, const double* lambda, int32_t mask_mode,
                  const uint8_t* mask,
                  double* d_gamma, double* d_rcv, double* d_eps) {
    if (n_src < 0 || n_rays < 0 || n_segs < 0 || n_rcv < 0 || n_freq < 0 || c <= 0) return -1;
    if (mask_mode == 2 && mask == NULL) return -1;
    cplx* Z = (cplx*)calloc((size_t)(n_faces > 0 ? n_faces : 1), sizeof(cplx));
    if (!Z) return -2;
    for (int64_t r = 0; r < n_rcv; ++r) d_rcv[3 * r] = d_rcv[3 * r + 1] = d_rcv[3 * r + 2] = 0.0;
    for (int32_t src = 0; src < n_src; ++src) {
        for (int32_t b = 0; b < n_freq; ++b) {
            const int64_t job = (int64_t)src * n_freq + b;
            const double omega = 2.0 * PI * freqs[b];
            const double k = omega / c;
            const double e = eps[job];
            const double al = alpha ? alpha[job] : 0.0;
            double deps_job = 0.0;
            for (int64_t r = 0; r < n_rcv; ++r) {
                const double* R = rcv + 3 * r;
                const cplx lam = lambda[2 * (job * n_rcv + r)] + I * lambda[2 * (job * n_rcv + r) + 1];
                for (int64_t i = 0; i < n_rays; ++i) {
                    if (ray_src[i] != src) continue;
                    const cplx weight = I * k * ray_w[i] / (8.0 * PI * PI);
                    for (int64_t j = ray_ptr[i]; j < ray_ptr[i + 1]; ++j) {
                        const double* a = seg_a + 3 * j;
                        const double* t = seg_t + 3 * j;
                        pair_geom g;
                        int inside = pair_geometry(R, a, t, seg_s0[j], seg_lo[j], seg_hi[j], &g);
                        cplx q;
                        cplx E = beam_exponent(omega, c, e, g.s, g.n2, &q);
                        int active = inside && creal(E) >= -gate_G;
                        if (mask_mode == 2) active = mask[(job * n_rcv + r) * n_segs + j];
                        if (!active) continue;
                        cplx q0 = -I * e;
                        cplx bare = weight * (q0 / q) * cexp(E) * exp(-al * g.s);   /* without prod Gamma */
                        cplx gp = face_product(face_ptr, face_ids, gamma, j);
                        cplx u = gp * bare;
                        /* receiver gradient */
                        double nvec[3] = {g.v[0] - g.sigma * t[0], g.v[1] - g.sigma * t[1], g.v[2] - g.sigma * t[2]};
                        cplx ct = I * k - 1.0 / q - 0.5 * I * k * g.n2 / (q * q) - al;
                        cplx cn = I * k / q;
                        for (int d = 0; d < 3; ++d) d_rcv[3 * r + d] += creal(lam * u * (ct * t[d] + cn * nvec[d]));
                        /* beam-parameter gradient */
                        deps_job += creal(lam * u * (1.0 / e + I / q - 0.5 * k * g.n2 / (q * q)));
                        /* reflection-coefficient gradient */
                        for (int64_t m = face_ptr[j]; m < face_ptr[j + 1]; ++m) {
                            int32_t f = face_ids[m];
                            /* count each distinct face once per segment */
                            int seen = 0;
                            for (int64_t mm = face_ptr[j]; mm < m; ++mm) seen |= (face_ids[mm] == f);
                            if (seen) continue;
                            Z[f] += lam * bare * face_product_deriv(face_ptr, face_ids, gamma, j, f);
                        }
                    }
                }
            }
            d_eps[job] = deps_job;
        }
    }
    for (int32_t f = 0; f < n_faces; ++f) {
        d_gamma[2 * f] = creal(Z[f]);
        d_gamma[2 * f + 1] = -cimag(Z[f]);
    }
    free(Z);
    return 0;
}

/*
 * Hand-derived adjoint for anisotropic beams (the field of gbso_forward_aniso),
 * dL = Re sum lambda dP.  With q_m = s - i eps_m, n_m = (R - a).e_m and the
 * amplitude sqrt(q01/q1) sqrt(q02/q2):
 *
 *   d ln u / dR    = t (ik - 1/(2 q1) - 1/(2 q2) - (ik/2)(n1^2/q1^2 + n2^2/q2^2)
 *                       - alpha) + (ik n1/q1) e1 + (ik n2/q2) e2
 *                    (ds/dR = t, dn_m/dR = e_m, d(1/q_m)/ds = -1/q_m^2,
 *                    d ln sqrt(q0m/qm)/ds = -1/(2 q_m))
 *   d ln u / deps_m = (1/eps_m + i/q_m)/2 - (k/2) n_m^2/q_m^2
 *                    (dq0m/deps_m = dq_m/deps_m = -i)
 *   dP / dGamma_f  as for isotropic beams (u without the coefficient product).
 *
 * With eps_1 = eps_2 = eps the two beam-parameter derivatives add up to the
 * isotropic d ln u/deps.  Outputs as gbso_backward, plus d_eps_e2[job].
 */
int gbso_backward_aniso(int32_t n_src, int64_t n_rays, const int64_t* ray_ptr, const double* ray_w,
                        const int32_t* ray_src, int64_t n_segs, const double* seg_a, const double* seg_t,
                        const double* seg_s0, const double* seg_lo, const double* seg_hi, const int64_t* face_ptr,
                        const int32_t* face_ids, int32_t n_faces, const double* gamma, int64_t n_rcv,
                        const double* rcv, int32_t n_freq, const double* freqs, const double* eps,
                        const double* alpha, double c, double gate_G, const double* eps_e2, const double* seg_e1,
                        const double* lambda, int32_t mask_mode, const uint8_t* mask, double* d_gamma,
                        double* d_rcv, double* d_eps, double* d_eps_e2) {
    if (n_src < 0 || n_rays < 0 || n_segs < 0 || n_rcv < 0 || n_freq < 0 || c <= 0) return -1;
    if (eps_e2 == NULL || (n_segs > 0 && seg_e1 == NULL)) return -1;
    if (mask_mode == 2 && mask == NULL) return -1;
    cplx* Z = (cplx*)calloc((size_t)(n_faces > 0 ? n_faces : 1), sizeof(cplx));
    if (!Z) return -2;
    for (int64_t r = 0; r < n_rcv; ++r) d_rcv[3 * r] = d_rcv[3 * r + 1] = d_rcv[3 * r + 2] = 0.0;
    for (int32_t src = 0; src < n_src; ++src) {
        for (int32_t b = 0; b < n_freq; ++b) {
            const int64_t job = (int64_t)src * n_freq + b;
            const double omega = 2.0 * PI * freqs[b];
            const double k = omega / c;
            const double p = 1.0 / c;
            const double e1 = eps[job], e2 = eps_e2[job];
            const double al = alpha ? alpha[job] : 0.0;
            double de1 = 0.0, de2 = 0.0;
            for (int64_t r = 0; r < n_rcv; ++r) {
                const double* R = rcv + 3 * r;
                const cplx lam = lambda[2 * (job * n_rcv + r)] + I * lambda[2 * (job * n_rcv + r) + 1];
                for (int64_t i = 0; i < n_rays; ++i) {
                    if (ray_src[i] != src) continue;
                    const cplx weight = I * k * ray_w[i] / (8.0 * PI * PI);
                    for (int64_t j = ray_ptr[i]; j < ray_ptr[i + 1]; ++j) {
                        const double* t = seg_t + 3 * j;
                        const double* f1 = seg_e1 + 3 * j;
                        pair_geom g;
                        const int inside = pair_geometry(R, seg_a + 3 * j, t, seg_s0[j], seg_lo[j], seg_hi[j], &g);
                        double n1, n2, f2[3];
                        frame_offsets(&g, t, f1, &n1, &n2, f2);
                        const cplx q01 = -I * e1, q02 = -I * e2;
                        const cplx q1 = q01 + g.s, q2 = q02 + g.s;
                        const cplx E = I * omega * (g.s / c + 0.5 * p * (n1 * n1 / q1 + n2 * n2 / q2));
                        int active = inside && creal(E) >= -gate_G;
                        if (mask_mode == 2) active = mask[(job * n_rcv + r) * n_segs + j];
                        if (!active) continue;
                        const cplx bare = weight * csqrt(q01 / q1) * csqrt(q02 / q2) * cexp(E) * exp(-al * g.s);
                        const cplx u = face_product(face_ptr, face_ids, gamma, j) * bare;
                        const cplx lu = lam * u;
                        const cplx ct = I * k - 0.5 / q1 - 0.5 / q2 - 0.5 * I * k * (n1 * n1 / (q1 * q1) +
                                        n2 * n2 / (q2 * q2)) - al;
                        const cplx c1 = I * k * n1 / q1, c2 = I * k * n2 / q2;
                        for (int d = 0; d < 3; ++d) d_rcv[3 * r + d] += creal(lu * (ct * t[d] + c1 * f1[d] + c2 * f2[d]));
                        de1 += creal(lu * (0.5 * (1.0 / e1 + I / q1) - 0.5 * k * n1 * n1 / (q1 * q1)));
                        de2 += creal(lu * (0.5 * (1.0 / e2 + I / q2) - 0.5 * k * n2 * n2 / (q2 * q2)));
                        for (int64_t m = face_ptr[j]; m < face_ptr[j + 1]; ++m) {
                            int32_t f = face_ids[m];
                            int seen = 0;
                            for (int64_t mm = face_ptr[j]; mm < m; ++mm) seen |= (face_ids[mm] == f);
                            if (seen) continue;
                            Z[f] += lam * bare * face_product_deriv(face_ptr, face_ids, gamma, j, f);
                        }
                    }
                }
            }
            d_eps[job] = de1;
            d_eps_e2[job] = de2;
        }
    }
    for (int32_t f = 0; f < n_faces; ++f) {
        d_gamma[2 * f] = creal(Z[f]);
        d_gamma[2 * f + 1] = -cimag(Z[f]);
    }
    free(Z);
    return 0;
}

/*
 * Pure-tone atmospheric attenuation coefficient in dB per metre (ISO 9613-1,
 * its Eqs. for the molar concentration of water vapour, the oxygen and
 * nitrogen relaxation frequencies and the attenuation), for frequency f (Hz),
 * air temperature temp_c (deg C), relative humidity rh (%) and pressure
 * p_atm (atmospheres).  The paper's runs use 20 deg C, 70 % and 1 atm.
 */
double gbso_air_absorption_db(double f, double temp_c, double rh, double p_atm) {
    const double T = temp_c + 273.15;       /* K */
    const double T0 = 293.15;               /* reference air temperature */
    const double T01 = 273.16;              /* triple-point isotherm */
    const double pa = p_atm;                /* pressure relative to 101.325 kPa */
    const double C = -6.8346 * pow(T01 / T, 1.261) + 4.6151;
    const double psat = pow(10.0, C);       /* saturation vapour pressure / reference */
    const double h = rh * psat / pa;        /* molar concentration of water vapour (%) */
    const double frO = pa * (24.0 + 4.04e4 * h * (0.02 + h) / (0.391 + h));
    const double frN = pa * pow(T / T0, -0.5) * (9.0 + 280.0 * h * exp(-4.170 * (pow(T / T0, -1.0 / 3.0) - 1.0)));
    const double f2 = f * f;
    return 8.686 * f2 *
           (1.84e-11 / pa * sqrt(T / T0) +
            pow(T / T0, -2.5) * (0.01275 * exp(-2239.1 / T) / (frO + f2 / frO) +
                                 0.1068 * exp(-3352.0 / T) / (frN + f2 / frN)));
}

int gbso_version(void) { return 3; }

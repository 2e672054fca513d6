/*
 * FP64 CPU oracle for QAOA max-cut state-vector simulation
 * (Lin, Wang, Tu, Hung, "Towards Optimizations of Quantum Circuit Simulation
 * for Solving Max-Cut Problems with QAOA", arXiv:2312.03019).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant
 * with the HIP library.
 *
 * It is deliberately the plain definition of what the simulator computes,
 * written out in double precision, with no blocking, fusion or reordering:
 *
 *   state    : 2^n complex amplitudes, index z, qubit q = bit q of z
 *              (the bit extraction (b >> i) & 1 of Algorithm 3).
 *   cut      : C(z) = sum over edges (u,v) of w_uv * [z_u != z_v], summed
 *              edge by edge in canonical (u<v, lexicographic) order.  This
 *              is the max-cut objective; Eq. UC_opt writes the cost layer
 *              through sum w (-1)^(z_u xor z_v) = W - 2 C(z).
 *   start    : every amplitude 2^(-n/2) (launch control, Section
 *              "Mathematical Optimizations"; equals H on every qubit).
 *   layer l  : cost   psi_z <- exp(-i gamma_l C(z)) psi_z   (diagonal form
 *                     of Eq. UC_opt, rotation compression, Algorithm 2)
 *              mixer  RX(2 beta_l) = exp(-i beta_l X_q) on every qubit q,
 *                     one qubit at a time (mixer layer of Algorithm 1).
 *   <C>      : sum_z |psi_z|^2 C(z), and the norm sum_z |psi_z|^2, both
 *              Neumaier-compensated over fixed chunks combined in order, so
 *              the result does not depend on the thread count.
 *   gradient : adjoint recurrence dE/dbeta_l = 2 Im <lam|B|phi>,
 *              dE/dgamma_l = 2 Im <lam|C|phi> with lam = (later gates)^dag C psi_p.
 *
 * The sign/scale convention (exp(-i gamma C), RX(2 beta)) differs from the
 * paper's printed one (exp(-i gamma/2 sum w Z Z), RX(beta)) by gamma -> -gamma
 * and beta -> beta/2 plus a global phase; the Python side offers the paper
 * form for a cross-check.
 *
 * All entry points return 0 on success, -1 on invalid input, -2 when memory
 * cannot be allocated.  Complex arrays are interleaved (re, im) doubles.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CHUNK 4096

/* Neumaier-compensated accumulator. */
typedef struct { double s, c; } ksum;
static void ks_add(ksum *k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static double ks_val(const ksum *k) { return k->s + k->c; }

static int check_graph(int n, int m, const int32_t *edges, const double *w) {
    if (n < 1 || n > 35 || m < 0) return -1;
    if (m > 0 && !edges) return -1;
    for (int e = 0; e < m; ++e) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) return -1;
        if (w && !isfinite(w[e])) return -1;
    }
    return 0;
}

/* C(z) for every z, by the per-edge definition. */
int oracle_cut_table(int n, int m, const int32_t *edges, const double *w, double *out) {
    if (check_graph(n, m, edges, w) || !out) return -1;
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) {
        double c = 0.0;
        for (int e = 0; e < m; ++e) {
            int u = edges[2 * e], v = edges[2 * e + 1];
            int cut = (int)(((z >> u) ^ (z >> v)) & 1);
            if (cut) c += w ? w[e] : 1.0;
        }
        out[z] = c;
    }
    return 0;
}

static void apply_cost(int64_t N, double *psi, const double *cut, double gamma) {
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) {
        double th = gamma * cut[z];
        double c = cos(th), s = -sin(th);           /* exp(-i th) */
        double re = psi[2 * z], im = psi[2 * z + 1];
        psi[2 * z] = re * c - im * s;
        psi[2 * z + 1] = re * s + im * c;
    }
}

/* exp(-i beta X_q) on one qubit: (a,b) -> (cos b a - i sin b b, -i sin b a + cos b b). */
static void apply_rx(int64_t N, double *psi, int q, double beta) {
    const int64_t bit = (int64_t)1 << q;
    const double c = cos(beta), s = sin(beta);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) {
        if (z & bit) continue;
        double *a = psi + 2 * z, *b = psi + 2 * (z | bit);
        double ar = a[0], ai = a[1], br = b[0], bi = b[1];
        a[0] = c * ar + s * bi;
        a[1] = c * ai - s * br;
        b[0] = s * ai + c * br;
        b[1] = -s * ar + c * bi;
    }
}

static int evolve_with_table(int n, const double *cut, int p, const double *gamma,
                             const double *beta, double *psi) {
    const int64_t N = (int64_t)1 << n;
    const double amp = pow(2.0, -0.5 * n);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) { psi[2 * z] = amp; psi[2 * z + 1] = 0.0; }
    for (int l = 0; l < p; ++l) {
        apply_cost(N, psi, cut, gamma[l]);
        for (int q = 0; q < n; ++q) apply_rx(N, psi, q, beta[l]);
    }
    return 0;
}

static int check_angles(int p, const double *gamma, const double *beta) {
    if (p < 0 || (p > 0 && (!gamma || !beta))) return -1;
    for (int l = 0; l < p; ++l)
        if (!isfinite(gamma[l]) || !isfinite(beta[l])) return -1;
    return 0;
}

/* Final state psi_p (2*2^n doubles). */
int oracle_evolve(int n, int m, const int32_t *edges, const double *w, int p,
                  const double *gamma, const double *beta, double *psi) {
    if (check_graph(n, m, edges, w) || check_angles(p, gamma, beta) || !psi) return -1;
    const int64_t N = (int64_t)1 << n;
    double *cut = (double *)malloc(sizeof(double) * N);
    if (!cut) return -2;
    oracle_cut_table(n, m, edges, w, cut);
    evolve_with_table(n, cut, p, gamma, beta, psi);
    free(cut);
    return 0;
}

/* sum over z of f(z) with fixed chunking: chunk sums in parallel, combined in order. */
static void chunked_sums(int64_t N, const double *psi, const double *cut,
                         double *e_out, double *norm_out) {
    int64_t nch = (N + CHUNK - 1) / CHUNK;
    double *pe = (double *)malloc(sizeof(double) * nch);
    double *pn = (double *)malloc(sizeof(double) * nch);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nch; ++k) {
        ksum se = {0, 0}, sn = {0, 0};
        int64_t hi = (k + 1) * CHUNK < N ? (k + 1) * CHUNK : N;
        for (int64_t z = k * CHUNK; z < hi; ++z) {
            double pr = psi[2 * z] * psi[2 * z] + psi[2 * z + 1] * psi[2 * z + 1];
            ks_add(&sn, pr);
            if (cut) ks_add(&se, pr * cut[z]);
        }
        pe[k] = ks_val(&se);
        pn[k] = ks_val(&sn);
    }
    ksum te = {0, 0}, tn = {0, 0};
    for (int64_t k = 0; k < nch; ++k) { ks_add(&te, pe[k]); ks_add(&tn, pn[k]); }
    if (e_out) *e_out = ks_val(&te);
    if (norm_out) *norm_out = ks_val(&tn);
    free(pe);
    free(pn);
}

/* <C> and norm of a given state (interleaved complex128) against a cut table. */
int oracle_expect(int n, const double *psi, const double *cut, double *e_out, double *norm_out) {
    if (n < 1 || n > 35 || !psi || !cut) return -1;
    chunked_sums((int64_t)1 << n, psi, cut, e_out, norm_out);
    return 0;
}

/* Evolve from |+>^n and return <C> and the norm (no state kept). */
int oracle_run_expect(int n, int m, const int32_t *edges, const double *w, int p,
                      const double *gamma, const double *beta, double *e_out, double *norm_out) {
    if (check_graph(n, m, edges, w) || check_angles(p, gamma, beta)) return -1;
    const int64_t N = (int64_t)1 << n;
    double *cut = (double *)malloc(sizeof(double) * N);
    double *psi = (double *)malloc(sizeof(double) * 2 * N);
    if (!cut || !psi) { free(cut); free(psi); return -2; }
    oracle_cut_table(n, m, edges, w, cut);
    evolve_with_table(n, cut, p, gamma, beta, psi);
    chunked_sums(N, psi, cut, e_out, norm_out);
    free(cut);
    free(psi);
    return 0;
}

/* Im <lam | X_q | phi>, summed over all qubits, compensated in fixed chunks. */
static double im_lam_B_phi(int n, const double *lam, const double *phi) {
    const int64_t N = (int64_t)1 << n;
    int64_t nch = (N + CHUNK - 1) / CHUNK;
    double *part = (double *)malloc(sizeof(double) * nch);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nch; ++k) {
        ksum s = {0, 0};
        int64_t hi = (k + 1) * CHUNK < N ? (k + 1) * CHUNK : N;
        for (int64_t z = k * CHUNK; z < hi; ++z) {
            for (int q = 0; q < n; ++q) {
                int64_t y = z ^ ((int64_t)1 << q);
                /* Im(conj(lam_z) phi_y) */
                ks_add(&s, lam[2 * z] * phi[2 * y + 1] - lam[2 * z + 1] * phi[2 * y]);
            }
        }
        part[k] = ks_val(&s);
    }
    ksum t = {0, 0};
    for (int64_t k = 0; k < nch; ++k) ks_add(&t, part[k]);
    free(part);
    return ks_val(&t);
}

/* Im <lam | C | phi>. */
static double im_lam_C_phi(int n, const double *lam, const double *phi, const double *cut) {
    const int64_t N = (int64_t)1 << n;
    int64_t nch = (N + CHUNK - 1) / CHUNK;
    double *part = (double *)malloc(sizeof(double) * nch);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nch; ++k) {
        ksum s = {0, 0};
        int64_t hi = (k + 1) * CHUNK < N ? (k + 1) * CHUNK : N;
        for (int64_t z = k * CHUNK; z < hi; ++z)
            ks_add(&s, cut[z] * (lam[2 * z] * phi[2 * z + 1] - lam[2 * z + 1] * phi[2 * z]));
        part[k] = ks_val(&s);
    }
    ksum t = {0, 0};
    for (int64_t k = 0; k < nch; ++k) ks_add(&t, part[k]);
    free(part);
    return ks_val(&t);
}

/*
 * <C> and its gradient with respect to every gamma_l and beta_l by the
 * adjoint recurrence: run forward to psi_p, set lam = C psi_p, then for
 * l = p..1 take dbeta_l = 2 Im<lam|B|phi> (B = sum_q X_q), undo mixer l on
 * both vectors, take dgamma_l = 2 Im<lam|C|phi>, undo cost l on both.
 */
int oracle_grad(int n, int m, const int32_t *edges, const double *w, int p,
                const double *gamma, const double *beta, double *e_out,
                double *dgamma, double *dbeta) {
    if (check_graph(n, m, edges, w) || check_angles(p, gamma, beta)) return -1;
    if (p > 0 && (!dgamma || !dbeta)) return -1;
    const int64_t N = (int64_t)1 << n;
    double *cut = (double *)malloc(sizeof(double) * N);
    double *phi = (double *)malloc(sizeof(double) * 2 * N);
    double *lam = (double *)malloc(sizeof(double) * 2 * N);
    if (!cut || !phi || !lam) { free(cut); free(phi); free(lam); return -2; }
    oracle_cut_table(n, m, edges, w, cut);
    evolve_with_table(n, cut, p, gamma, beta, phi);
    chunked_sums(N, phi, cut, e_out, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; ++z) {
        lam[2 * z] = cut[z] * phi[2 * z];
        lam[2 * z + 1] = cut[z] * phi[2 * z + 1];
    }
    for (int l = p - 1; l >= 0; --l) {
        dbeta[l] = 2.0 * im_lam_B_phi(n, lam, phi);
        for (int q = 0; q < n; ++q) {
            apply_rx(N, phi, q, -beta[l]);
            apply_rx(N, lam, q, -beta[l]);
        }
        dgamma[l] = 2.0 * im_lam_C_phi(n, lam, phi, cut);
        apply_cost(N, phi, cut, -gamma[l]);
        apply_cost(N, lam, cut, -gamma[l]);
    }
    free(cut);
    free(phi);
    free(lam);
    return 0;
}

/* F = |<a|b>|^2 / (<a|a><b|b>), interleaved complex128 inputs. */
int oracle_fidelity(int n, const double *a, const double *b, double *f_out) {
    if (n < 1 || n > 35 || !a || !b || !f_out) return -1;
    const int64_t N = (int64_t)1 << n;
    int64_t nch = (N + CHUNK - 1) / CHUNK;
    double *pr = (double *)malloc(sizeof(double) * nch);
    double *pi = (double *)malloc(sizeof(double) * nch);
    double *pa = (double *)malloc(sizeof(double) * nch);
    double *pb = (double *)malloc(sizeof(double) * nch);
    if (!pr || !pi || !pa || !pb) { free(pr); free(pi); free(pa); free(pb); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nch; ++k) {
        ksum sr = {0, 0}, si = {0, 0}, sa = {0, 0}, sb = {0, 0};
        int64_t hi = (k + 1) * CHUNK < N ? (k + 1) * CHUNK : N;
        for (int64_t z = k * CHUNK; z < hi; ++z) {
            double ar = a[2 * z], ai = a[2 * z + 1], br = b[2 * z], bi = b[2 * z + 1];
            ks_add(&sr, ar * br + ai * bi);   /* Re conj(a) b */
            ks_add(&si, ar * bi - ai * br);   /* Im conj(a) b */
            ks_add(&sa, ar * ar + ai * ai);
            ks_add(&sb, br * br + bi * bi);
        }
        pr[k] = ks_val(&sr); pi[k] = ks_val(&si); pa[k] = ks_val(&sa); pb[k] = ks_val(&sb);
    }
    ksum tr = {0, 0}, ti = {0, 0}, ta = {0, 0}, tb = {0, 0};
    for (int64_t k = 0; k < nch; ++k) {
        ks_add(&tr, pr[k]); ks_add(&ti, pi[k]); ks_add(&ta, pa[k]); ks_add(&tb, pb[k]);
    }
    double re = ks_val(&tr), im = ks_val(&ti);
    *f_out = (re * re + im * im) / (ks_val(&ta) * ks_val(&tb));
    free(pr); free(pi); free(pa); free(pb);
    return 0;
}

/* One amplitude of the depth-1 state, psi_z = <z| exp(-i beta B) exp(-i gamma C) |+>^n,
 * by its definition as a sum over the basis states x.  The mixer is the tensor
 * product of exp(-i beta X) on every qubit, whose matrix element <z_q|.|x_q> is
 * cos(beta) when z_q = x_q and -i sin(beta) otherwise, so
 *   psi_z = 2^(-n/2) sum_x cos(beta)^(n-d) (-i sin(beta))^d exp(-i gamma C(x)),
 * d = the number of qubits where x and z differ.  C(x) by the per-edge
 * definition.  Fixed chunks summed in parallel (Neumaier), combined in order.
 * out: (re, im). */
int oracle_amplitude_p1(int n, int m, const int32_t *edges, const double *w, double gamma,
                        double beta, int64_t z, double *out) {
    if (check_graph(n, m, edges, w) || !out || !isfinite(gamma) || !isfinite(beta)) return -1;
    const int64_t N = (int64_t)1 << n;
    if (z < 0 || z >= N) return -1;
    double fre[65], fim[65];
    const double cb = cos(beta), sb = sin(beta);
    for (int d = 0; d <= n; ++d) {
        const double mag = pow(cb, n - d) * pow(sb, d);
        /* (-i)^d */
        const double pr[4] = {1.0, 0.0, -1.0, 0.0}, pi[4] = {0.0, -1.0, 0.0, 1.0};
        fre[d] = mag * pr[d & 3];
        fim[d] = mag * pi[d & 3];
    }
    const int64_t nch = (N + CHUNK - 1) / CHUNK;
    double *pre = (double *)malloc(sizeof(double) * nch), *pim = (double *)malloc(sizeof(double) * nch);
    if (!pre || !pim) { free(pre); free(pim); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nch; ++k) {
        ksum sr = {0, 0}, si = {0, 0};
        const int64_t end = (k + 1) * CHUNK < N ? (k + 1) * CHUNK : N;
        for (int64_t x = k * CHUNK; x < end; ++x) {
            double c = 0.0;
            for (int e = 0; e < m; ++e) {
                int u = edges[2 * e], v = edges[2 * e + 1];
                if (((x >> u) ^ (x >> v)) & 1) c += w ? w[e] : 1.0;
            }
            const double th = gamma * c;
            const double er = cos(th), ei = -sin(th);
            const int d = __builtin_popcountll((uint64_t)(x ^ z));
            ks_add(&sr, fre[d] * er - fim[d] * ei);
            ks_add(&si, fre[d] * ei + fim[d] * er);
        }
        pre[k] = ks_val(&sr);
        pim[k] = ks_val(&si);
    }
    ksum tr = {0, 0}, ti = {0, 0};
    for (int64_t k = 0; k < nch; ++k) { ks_add(&tr, pre[k]); ks_add(&ti, pim[k]); }
    const double amp = sqrt(ldexp(1.0, -n));   /* 2^(-n/2) */
    out[0] = amp * ks_val(&tr);
    out[1] = amp * ks_val(&ti);
    free(pre); free(pim);
    return 0;
}

/* Threads OpenMP will use (for reporting the CPU baseline's core count). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

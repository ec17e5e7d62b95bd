/*
 * plv_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, FP64 CPU reference for what the PLV hot path computes.  Only
 * the tests, the smoke check and the bench's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the HIP library.
 *
 * What it follows (Bruna, Maestu, Pereda, "Phase Locking Value revisited"):
 *   - analytic signal (Section II.A, Eq. 3): z = x_BP + i*Hilbert{x_BP}, built
 *     here as the DFT-domain construction (one-sided spectrum weights h_k) with
 *     plain O(T^2) DFT sums, no FFT; the band-pass x_BP either a DFT-bin mask
 *     or a forward-backward FIR (Section III names one, without its design);
 *   - instantaneous phase (Eq. 3 and the Appendix's first listing): the angle
 *     of z, atan2(Im z, Re z); an exact zero z gets phase 0;
 *   - PLV over time (Section II.A, Eq. 2): for each pair, the mean over t of
 *     exp(i(phase_i(t) - phase_j(t))), one complex exponential per
 *     pair-sample, i.e. the original per-pair formulation that the paper's
 *     matrix form (Eqs. 5-7) rewrites;
 *   - iPLV (Section II.C, Eq. 13) and ciPLV (Eq. 14) from the same mean;
 *   - coherency (Section II.B, Eq. 12): amplitude-weighted cross sums over
 *     the per-row powers; coherence is its magnitude, and the imaginary and
 *     corrected imaginary coherency follow the iPLV / ciPLV forms;
 *   - the gradient of a loss on these metrics, derived in angle space
 *     (d mean / d phase), chained through atan2 and the linear analytic-signal
 *     map.  Not in the paper; it checks the library's adjoint.
 *
 * Sums run in plain FP64 in sample order.  Threads split independent rows or
 * pairs only; they never reorder a sum.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Spectral weights of the analytic signal                                    */
/* ------------------------------------------------------------------------- */

/* One-sided spectrum weights of the discrete analytic signal (Marple, IEEE TSP
 * 47(9), 1999): h_0 = 1, h_k = 2 for 0 < k < T/2, h_{T/2} = 1 when T is even,
 * 0 for the negative-frequency bins. */
void oracle_mask_plain(int64_t t, double *h)
{
    for (int64_t k = 0; k < t; ++k) {
        if (k == 0)
            h[k] = 1.0;
        else if (2 * k < t)
            h[k] = 2.0;
        else if (2 * k == t)
            h[k] = 1.0;
        else
            h[k] = 0.0;
    }
}

/* Band-pass analytic signal (Eq. 3 with a brick-wall pass band): weight 2 on the
 * positive-frequency bins whose frequency k*fs/T lies in [flo, fhi], both ends
 * included; DC, Nyquist and everything else get 0. */
void oracle_mask_band(int64_t t, double fs, double flo, double fhi, double *h)
{
    for (int64_t k = 0; k < t; ++k) {
        double f = (double)k * fs / (double)t;
        int positive = (k > 0) && (2 * k < t);
        h[k] = (positive && f >= flo && f <= fhi) ? 2.0 : 0.0;
    }
}

/* FIR band-pass applied forward and backward (the paper's filtering before
 * the Hilbert transform, Section III; its design is not given there, so this
 * is the build's own definition).  Taps: the ideal band-pass impulse response
 * between flo and fhi (Hz, sampling rate fs) sampled at n = m - L/2,
 * m = 0..L (L even, L + 1 taps), times the symmetric Hamming window
 * 0.54 - 0.46 cos(2 pi m / L), then scaled to unit gain at the band centre
 * (flo + fhi) / 2.  Returns 0, or -1 for an odd or non-positive order. */
int oracle_fir_taps(int64_t order, double fs, double flo, double fhi, double *taps)
{
    if (order <= 0 || (order & 1))
        return -1;
    const double a = flo / fs, b = fhi / fs;  /* cycles per sample */
    const double half = (double)(order / 2);
    for (int64_t m = 0; m <= order; ++m) {
        const double n = (double)m - half;
        const double ideal = (m == order / 2) ? 2.0 * (b - a)
                                              : (sin(2.0 * M_PI * b * n) - sin(2.0 * M_PI * a * n)) / (M_PI * n);
        const double w = 0.54 - 0.46 * cos(2.0 * M_PI * (double)m / (double)order);
        taps[m] = ideal * w;
    }
    /* gain at the centre frequency: the taps are symmetric about L/2 */
    const double fc = 0.5 * (a + b);
    double g = 0.0;
    for (int64_t m = 0; m <= order; ++m)
        g += taps[m] * cos(2.0 * M_PI * fc * ((double)m - half));
    for (int64_t m = 0; m <= order; ++m)
        taps[m] /= g;
    return 0;
}

/* Zero-phase gain of that filter on the T-point DFT grid: forward then
 * backward filtering multiplies bin k by |H(exp(2 pi i k / T))|^2, with
 * H(e^{iw}) = sum_m taps[m] e^{-i w m} summed directly (angle index k m mod T).
 * Returns 0, or -1 for a bad order or an allocation failure. */
int oracle_fir_power(int64_t t, double fs, double flo, double fhi, int64_t order, double *p)
{
    double *taps = (double *)malloc(sizeof(double) * (size_t)(order + 1));
    if (!taps || oracle_fir_taps(order, fs, flo, fhi, taps)) {
        free(taps);
        return -1;
    }
    for (int64_t k = 0; k < t; ++k) {
        double re = 0.0, im = 0.0;
        for (int64_t m = 0; m <= order; ++m) {
            const double ang = 2.0 * M_PI * (double)((k * m) % t) / (double)t;
            re += taps[m] * cos(ang);
            im -= taps[m] * sin(ang);
        }
        p[k] = re * re + im * im;
    }
    free(taps);
    return 0;
}

/* Analytic signal of the FIR-filtered row: the one-sided weights above times
 * the zero-phase gain.  Returns 0 or -1 as oracle_fir_power. */
int oracle_mask_fir(int64_t t, double fs, double flo, double fhi, int64_t order, double *h)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)t);
    if (!p || oracle_fir_power(t, fs, flo, fhi, order, p)) {
        free(p);
        return -1;
    }
    oracle_mask_plain(t, h);
    for (int64_t k = 0; k < t; ++k)
        h[k] *= p[k];
    free(p);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Plain-DFT spectral filter:  out = IDFT( h .* DFT(in) )                     */
/* ------------------------------------------------------------------------- */

struct dft_job {
    const double *xr, *xi;  /* input rows (xi may be NULL: real input) */
    int64_t ldx;
    double *zr, *zi;        /* output rows */
    int64_t ldz;
    int64_t t;
    const double *h;
    const double *cs, *sn;  /* cos / sin of 2*pi*m/T, m = 0..T-1 */
    int64_t row0, row1;
};

static void dft_filter_row(const struct dft_job *jb, int64_t row, double *xre, double *xim)
{
    const int64_t t = jb->t;
    const double *xr = jb->xr + row * jb->ldx;
    const double *xi = jb->xi ? jb->xi + row * jb->ldx : NULL;
    /* forward DFT: X_k = sum_s x_s exp(-2 pi i k s / T) */
    for (int64_t k = 0; k < t; ++k) {
        double ar = 0.0, ai = 0.0;
        if (jb->h[k] != 0.0) {
            for (int64_t s = 0; s < t; ++s) {
                int64_t m = (k * s) % t;
                double c = jb->cs[m], sn = jb->sn[m];
                double vr = xr[s], vi = xi ? xi[s] : 0.0;
                /* (vr + i vi) * (c - i sn) */
                ar += vr * c + vi * sn;
                ai += vi * c - vr * sn;
            }
        }
        xre[k] = jb->h[k] * ar;
        xim[k] = jb->h[k] * ai;
    }
    /* inverse DFT: z_s = (1/T) sum_k Y_k exp(+2 pi i k s / T) */
    double *zr = jb->zr + row * jb->ldz, *zi = jb->zi + row * jb->ldz;
    for (int64_t s = 0; s < t; ++s) {
        double ar = 0.0, ai = 0.0;
        for (int64_t k = 0; k < t; ++k) {
            if (jb->h[k] == 0.0)
                continue;
            int64_t m = (k * s) % t;
            double c = jb->cs[m], sn = jb->sn[m];
            /* (xre + i xim) * (c + i sn) */
            ar += xre[k] * c - xim[k] * sn;
            ai += xre[k] * sn + xim[k] * c;
        }
        zr[s] = ar / (double)t;
        zi[s] = ai / (double)t;
    }
}

static void *dft_worker(void *arg)
{
    struct dft_job *jb = (struct dft_job *)arg;
    double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)jb->t);
    if (!buf)
        return (void *)1;
    for (int64_t r = jb->row0; r < jb->row1; ++r)
        dft_filter_row(jb, r, buf, buf + jb->t);
    free(buf);
    return NULL;
}

/* For each of `nrows` rows: z = IDFT(h .* DFT(x)), x = xr + i*xi (xi may be
 * NULL for real input).  Rows are split across `nthreads` threads.
 * Returns 0 on success, nonzero on allocation failure. */
int oracle_spectral_filter(const double *xr, const double *xi, int64_t ldx, int64_t nrows, int64_t t,
                           const double *h, double *zr, double *zi, int64_t ldz, int nthreads)
{
    if (t <= 0 || nrows <= 0)
        return 0;
    double *cs = (double *)malloc(sizeof(double) * (size_t)t);
    double *sn = (double *)malloc(sizeof(double) * (size_t)t);
    if (!cs || !sn) {
        free(cs);
        free(sn);
        return 1;
    }
    for (int64_t m = 0; m < t; ++m) {
        double a = 2.0 * M_PI * (double)m / (double)t;
        cs[m] = cos(a);
        sn[m] = sin(a);
    }
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > nrows)
        nthreads = (int)nrows;
    struct dft_job *jobs = (struct dft_job *)calloc((size_t)nthreads, sizeof(struct dft_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    int rc = 0;
    if (!jobs || !th) {
        rc = 1;
        goto done;
    }
    for (int w = 0; w < nthreads; ++w) {
        struct dft_job *jb = &jobs[w];
        jb->xr = xr;
        jb->xi = xi;
        jb->ldx = ldx;
        jb->zr = zr;
        jb->zi = zi;
        jb->ldz = ldz;
        jb->t = t;
        jb->h = h;
        jb->cs = cs;
        jb->sn = sn;
        jb->row0 = nrows * w / nthreads;
        jb->row1 = nrows * (w + 1) / nthreads;
        pthread_create(&th[w], NULL, dft_worker, jb);
    }
    for (int w = 0; w < nthreads; ++w) {
        void *ret = NULL;
        pthread_join(th[w], &ret);
        if (ret)
            rc = 1;
    }
done:
    free(jobs);
    free(th);
    free(cs);
    free(sn);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Instantaneous phase                                                        */
/* ------------------------------------------------------------------------- */

/* phase = angle(z) = atan2(Im z, Re z); an exact zero (either zero sign) gets 0. */
void oracle_phase(const double *zr, const double *zi, int64_t count, double *phi)
{
    for (int64_t q = 0; q < count; ++q) {
        if (zr[q] == 0.0 && zi[q] == 0.0)
            phi[q] = 0.0;
        else
            phi[q] = atan2(zi[q], zr[q]);
    }
}

/* ------------------------------------------------------------------------- */
/* Per-pair mean of exp(i * phase difference)  (Eq. 2)                        */
/* ------------------------------------------------------------------------- */

struct pair_job {
    const double *phi;
    int64_t ld, t;
    const int64_t *pi, *pj;
    double *gre, *gim;
    int64_t p0, p1;
};

static void *pair_worker(void *arg)
{
    struct pair_job *jb = (struct pair_job *)arg;
    for (int64_t p = jb->p0; p < jb->p1; ++p) {
        const double *a = jb->phi + jb->pi[p] * jb->ld;
        const double *b = jb->phi + jb->pj[p] * jb->ld;
        double sr = 0.0, si = 0.0;
        for (int64_t s = 0; s < jb->t; ++s) {
            double d = a[s] - b[s];
            sr += cos(d);
            si += sin(d);
        }
        jb->gre[p] = sr / (double)jb->t;
        jb->gim[p] = si / (double)jb->t;
    }
    return NULL;
}

/* G[p] = (1/T) sum_t exp(i (phi[pi[p]](t) - phi[pj[p]](t))) for each listed pair.
 * phi is [rows][ld] with T valid samples per row. */
void oracle_pair_means(const double *phi, int64_t ld, int64_t t, const int64_t *pi, const int64_t *pj,
                       int64_t npairs, double *gre, double *gim, int nthreads)
{
    if (npairs <= 0)
        return;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > npairs)
        nthreads = (int)npairs;
    struct pair_job jobs[256];
    pthread_t th[256];
    if (nthreads > 256)
        nthreads = 256;
    for (int w = 0; w < nthreads; ++w) {
        jobs[w].phi = phi;
        jobs[w].ld = ld;
        jobs[w].t = t;
        jobs[w].pi = pi;
        jobs[w].pj = pj;
        jobs[w].gre = gre;
        jobs[w].gim = gim;
        jobs[w].p0 = npairs * w / nthreads;
        jobs[w].p1 = npairs * (w + 1) / nthreads;
        pthread_create(&th[w], NULL, pair_worker, &jobs[w]);
    }
    for (int w = 0; w < nthreads; ++w)
        pthread_join(th[w], NULL);
}

/* ------------------------------------------------------------------------- */
/* Metrics  (Eq. 2 magnitude, Eq. 13, Eq. 14)                                 */
/* ------------------------------------------------------------------------- */

/* plv = |G|, iplv = |Im G|, ciplv = |Im G| / sqrt(1 - (Re G)^2), with the
 * radicand taken as (1 - Re)(1 + Re); ciplv = 0 when the radicand is <= 0. */
void oracle_metrics(const double *gre, const double *gim, int64_t count, double *plv, double *iplv,
                    double *ciplv)
{
    for (int64_t q = 0; q < count; ++q) {
        double r = gre[q], m = gim[q];
        double d = (1.0 - r) * (1.0 + r);
        if (plv)
            plv[q] = hypot(r, m);
        if (iplv)
            iplv[q] = fabs(m);
        if (ciplv)
            ciplv[q] = d > 0.0 ? fabs(m) / sqrt(d) : 0.0;
    }
}

/* ------------------------------------------------------------------------- */
/* Coherency (Section II.B, Eq. 12)                                           */
/* ------------------------------------------------------------------------- */

/* Complex coherency of each listed pair of complex rows (Fourier coefficients
 * over trials or windows, or analytic signals over time):
 *   C[p] = sum_t X_a(t) conj(X_b(t)) / sqrt(sum_t |X_a(t)|^2 * sum_t |X_b(t)|^2)
 * with (a, b) = (pi[p], pj[p]); its magnitude is the coherence of Eq. 12.  A
 * pair with an all-zero row has no defined coherency and gets C = 0.  Sums in
 * FP64 in sample order. */
struct coh_job {
    const double *zr, *zi;
    int64_t ld, t;
    const int64_t *pi, *pj;
    double *cre, *cim;
    int64_t p0, p1;
};

static double row_power(const double *zr, const double *zi, int64_t t)
{
    double s = 0.0;
    for (int64_t k = 0; k < t; ++k)
        s += zr[k] * zr[k] + zi[k] * zi[k];
    return s;
}

static void *coh_worker(void *arg)
{
    struct coh_job *jb = (struct coh_job *)arg;
    for (int64_t p = jb->p0; p < jb->p1; ++p) {
        const double *ar = jb->zr + jb->pi[p] * jb->ld, *ai = jb->zi + jb->pi[p] * jb->ld;
        const double *br = jb->zr + jb->pj[p] * jb->ld, *bi = jb->zi + jb->pj[p] * jb->ld;
        double sr = 0.0, si = 0.0;
        for (int64_t k = 0; k < jb->t; ++k) {
            /* X_a conj(X_b) = (ar + i ai)(br - i bi) */
            sr += ar[k] * br[k] + ai[k] * bi[k];
            si += ai[k] * br[k] - ar[k] * bi[k];
        }
        const double pa = row_power(ar, ai, jb->t), pb = row_power(br, bi, jb->t);
        const double den = sqrt(pa) * sqrt(pb);
        jb->cre[p] = den > 0.0 ? sr / den : 0.0;
        jb->cim[p] = den > 0.0 ? si / den : 0.0;
    }
    return NULL;
}

void oracle_coherency(const double *zr, const double *zi, int64_t ld, int64_t t, const int64_t *pi,
                      const int64_t *pj, int64_t npairs, double *cre, double *cim, int nthreads)
{
    if (npairs <= 0)
        return;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > npairs)
        nthreads = (int)npairs;
    if (nthreads > 256)
        nthreads = 256;
    struct coh_job jobs[256];
    pthread_t th[256];
    for (int w = 0; w < nthreads; ++w) {
        jobs[w].zr = zr;
        jobs[w].zi = zi;
        jobs[w].ld = ld;
        jobs[w].t = t;
        jobs[w].pi = pi;
        jobs[w].pj = pj;
        jobs[w].cre = cre;
        jobs[w].cim = cim;
        jobs[w].p0 = npairs * w / nthreads;
        jobs[w].p1 = npairs * (w + 1) / nthreads;
        pthread_create(&th[w], NULL, coh_worker, &jobs[w]);
    }
    for (int w = 0; w < nthreads; ++w)
        pthread_join(th[w], NULL);
}

/* ------------------------------------------------------------------------- */
/* Gradient (angle space)                                                     */
/* ------------------------------------------------------------------------- */

/* Per pair: given dL/dplv, dL/diplv, dL/dciplv (already combined over (i,j) and
 * (j,i)), return dL/dRe G and dL/dIm G.  sign(0) = 0; the PLV term is dropped
 * where |G| = 0 and the ciPLV term where the radicand is <= 0. */
void oracle_metric_adjoint(const double *gre, const double *gim, const double *gp, const double *gi,
                           const double *gc, int64_t count, double *dre, double *dim)
{
    for (int64_t q = 0; q < count; ++q) {
        double r = gre[q], m = gim[q];
        double sgn = (m > 0.0) ? 1.0 : ((m < 0.0) ? -1.0 : 0.0);
        double ar = 0.0, am = 0.0;
        if (gp) {
            double p = hypot(r, m);
            if (p > 0.0) {
                ar += gp[q] * r / p;
                am += gp[q] * m / p;
            }
        }
        if (gi)
            am += gi[q] * sgn;
        if (gc) {
            double d = (1.0 - r) * (1.0 + r);
            if (d > 0.0) {
                double s = sqrt(d);
                am += gc[q] * sgn / s;
                ar += gc[q] * fabs(m) * r / (s * d);
            }
        }
        dre[q] = ar;
        dim[q] = am;
    }
}

struct grad_job {
    const double *phi;
    int64_t ld, n, t;
    const double *dre, *dim; /* [n][n]: entry (a,b), a < b, holds the pair's dL/dRe G, dL/dIm G */
    double *dphi;
    int64_t ldd;
    int64_t r0, r1;
};

static void *grad_worker(void *arg)
{
    struct grad_job *jb = (struct grad_job *)arg;
    const int64_t n = jb->n, t = jb->t;
    const double inv_t = 1.0 / (double)t;
    for (int64_t i = jb->r0; i < jb->r1; ++i) {
        double *out = jb->dphi + i * jb->ldd;
        for (int64_t s = 0; s < t; ++s)
            out[s] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            /* pair (a, b) with a < b; G_ab = mean exp(i(phi_a - phi_b)).
             * dG_ab/dphi_a(t) = (i/T) exp(i d), dG_ab/dphi_b(t) = -(i/T) exp(i d). */
            int64_t a = i < j ? i : j, b = i < j ? j : i;
            double gr = jb->dre[a * n + b], gm = jb->dim[a * n + b];
            if (gr == 0.0 && gm == 0.0)
                continue;
            double sign = (i == a) ? 1.0 : -1.0;
            const double *pa = jb->phi + a * jb->ld, *pb = jb->phi + b * jb->ld;
            for (int64_t s = 0; s < t; ++s) {
                double d = pa[s] - pb[s];
                /* dL/dphi = gr * dRe/dphi + gm * dIm/dphi, with
                 * d(cos d)/dphi_a = -sin d, d(sin d)/dphi_a = cos d */
                out[s] += sign * (gr * (-sin(d)) + gm * cos(d)) * inv_t;
            }
        }
    }
    return NULL;
}

/* dL/dphi of the listed rows only (rows[r] -> dphi row r), same sums as
 * oracle_phase_grad. */
struct grad_rows_job {
    struct grad_job base;
    const int64_t *rows;
};

static void *grad_rows_worker(void *arg)
{
    struct grad_rows_job *rj = (struct grad_rows_job *)arg;
    struct grad_job *jb = &rj->base;
    const int64_t n = jb->n, t = jb->t;
    const double inv_t = 1.0 / (double)t;
    for (int64_t r = jb->r0; r < jb->r1; ++r) {
        const int64_t i = rj->rows[r];
        double *out = jb->dphi + r * jb->ldd;
        for (int64_t s = 0; s < t; ++s)
            out[s] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            int64_t a = i < j ? i : j, b = i < j ? j : i;
            double gr = jb->dre[a * n + b], gm = jb->dim[a * n + b];
            if (gr == 0.0 && gm == 0.0)
                continue;
            double sign = (i == a) ? 1.0 : -1.0;
            const double *pa = jb->phi + a * jb->ld, *pb = jb->phi + b * jb->ld;
            for (int64_t s = 0; s < t; ++s) {
                double d = pa[s] - pb[s];
                out[s] += sign * (gr * (-sin(d)) + gm * cos(d)) * inv_t;
            }
        }
    }
    return NULL;
}

void oracle_phase_grad_rows(const double *phi, int64_t ld, int64_t n, int64_t t, const double *dre,
                            const double *dim, const int64_t *rows, int64_t nrows, double *dphi, int64_t ldd,
                            int nthreads)
{
    if (nrows <= 0)
        return;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > nrows)
        nthreads = (int)nrows;
    if (nthreads > 256)
        nthreads = 256;
    struct grad_rows_job jobs[256];
    pthread_t th[256];
    for (int w = 0; w < nthreads; ++w) {
        jobs[w].base.phi = phi;
        jobs[w].base.ld = ld;
        jobs[w].base.n = n;
        jobs[w].base.t = t;
        jobs[w].base.dre = dre;
        jobs[w].base.dim = dim;
        jobs[w].base.dphi = dphi;
        jobs[w].base.ldd = ldd;
        jobs[w].base.r0 = nrows * w / nthreads;
        jobs[w].base.r1 = nrows * (w + 1) / nthreads;
        jobs[w].rows = rows;
        pthread_create(&th[w], NULL, grad_rows_worker, &jobs[w]);
    }
    for (int w = 0; w < nthreads; ++w)
        pthread_join(th[w], NULL);
}

/* dL/dphi for every row, from per-pair dL/dRe G and dL/dIm G stored in the
 * upper triangle of [n][n] arrays. */
void oracle_phase_grad(const double *phi, int64_t ld, int64_t n, int64_t t, const double *dre, const double *dim,
                       double *dphi, int64_t ldd, int nthreads)
{
    if (n <= 0)
        return;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > n)
        nthreads = (int)n;
    if (nthreads > 256)
        nthreads = 256;
    struct grad_job jobs[256];
    pthread_t th[256];
    for (int w = 0; w < nthreads; ++w) {
        jobs[w].phi = phi;
        jobs[w].ld = ld;
        jobs[w].n = n;
        jobs[w].t = t;
        jobs[w].dre = dre;
        jobs[w].dim = dim;
        jobs[w].dphi = dphi;
        jobs[w].ldd = ldd;
        jobs[w].r0 = n * w / nthreads;
        jobs[w].r1 = n * (w + 1) / nthreads;
        pthread_create(&th[w], NULL, grad_worker, &jobs[w]);
    }
    for (int w = 0; w < nthreads; ++w)
        pthread_join(th[w], NULL);
}

/* Chain dL/dphase back to z through phase = atan2(Im z, Re z):
 * dphase/dRe z = -Im z / |z|^2, dphase/dIm z = Re z / |z|^2; zero at z = 0. */
void oracle_phase_to_z(const double *zr, const double *zi, const double *dphi, int64_t count, double *dzr,
                       double *dzi)
{
    for (int64_t q = 0; q < count; ++q) {
        double r2 = zr[q] * zr[q] + zi[q] * zi[q];
        if (r2 == 0.0) {
            dzr[q] = 0.0;
            dzi[q] = 0.0;
        } else {
            dzr[q] = -dphi[q] * zi[q] / r2;
            dzi[q] = dphi[q] * zr[q] / r2;
        }
    }
}

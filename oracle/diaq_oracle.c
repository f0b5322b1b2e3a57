/*
 * diaq_oracle.c -- plain CPU reference for the DiaQ hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this code.  It shares nothing
 * (no header, no table, no helper) with the HIP library and never calls it.
 *
 * Everything here is written for obviousness, not speed: fp64 throughout,
 * no blocking, no fusion, plain loops.  OpenMP only splits independent
 * outer iterations across threads; it changes no arithmetic.
 *
 * Complex numbers are interleaved (re, im) pairs of doubles.  Qubit q is
 * bit q of an amplitude index (little-endian).
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <omp.h>

/* Thread count of the parallel loops below (the CPU baseline is timed on
 * all host cores and on one); no effect on any result. */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* State evolution by amplitude-index bit manipulation                 */
/* ------------------------------------------------------------------ */

/*
 * psi <- (I_above (x) M (x) I_below) psi for one gate (Sec. II-C), where M
 * is a dim x dim matrix (dim = 2^k) acting on the qubits targets[0..k)
 * (targets[0] = local bit 0) and applied only where every qubit in
 * controls[0..nc) is 1.
 *
 * For every index b whose target bits are all 0 and whose control bits are
 * all 1, the dim amplitudes psi[b + scatter(r)] form a small vector v; it
 * is replaced by M v.  scatter(r) places bit j of r at qubit targets[j].
 */
void orc_apply_gate(double *psi, int n, const double *m, int k,
                    const int *targets, int nc, const int *controls)
{
    const int64_t N = (int64_t)1 << n;
    const int dim = 1 << k;
    int64_t tmask = 0, cmask = 0;
    int64_t sc[8];
    for (int j = 0; j < k; j++) tmask |= (int64_t)1 << targets[j];
    for (int j = 0; j < nc; j++) cmask |= (int64_t)1 << controls[j];
    for (int r = 0; r < dim; r++) {
        int64_t s = 0;
        for (int j = 0; j < k; j++)
            if ((r >> j) & 1) s |= (int64_t)1 << targets[j];
        sc[r] = s;
    }
#pragma omp parallel for schedule(static) if (N > 32768)
    for (int64_t b = 0; b < N; b++) {
        if ((b & tmask) != 0 || (b & cmask) != cmask) continue;
        double vr[8], vi[8];
        for (int r = 0; r < dim; r++) {
            vr[r] = psi[2 * (b + sc[r])];
            vi[r] = psi[2 * (b + sc[r]) + 1];
        }
        for (int r = 0; r < dim; r++) {
            double ar = 0.0, ai = 0.0;
            for (int c = 0; c < dim; c++) {
                const double mr = m[2 * (r * dim + c)];
                const double mi = m[2 * (r * dim + c) + 1];
                ar += mr * vr[c] - mi * vi[c];
                ai += mr * vi[c] + mi * vr[c];
            }
            psi[2 * (b + sc[r])] = ar;
            psi[2 * (b + sc[r]) + 1] = ai;
        }
    }
}

/* ------------------------------------------------------------------ */
/* DiaQ sparse matrix-vector product, from the format's definition      */
/* ------------------------------------------------------------------ */

/*
 * y <- A x for a DiaQ matrix of dimension N (Sec. IV): diagonal k has
 * index d = offsets[k] (column - row) and stores the N - |d| elements
 * A[t + max(0,-d), t + max(0,d)], t = 0 .. N-|d|-1, from element starts[k]
 * of vals.  So A[i, i+d] is element i - max(0,-d) of diagonal k, and
 *
 *     y[i] = sum over k with 0 <= i + d_k < N of  A[i, i+d_k] * x[i+d_k],
 *
 * taken one row at a time, diagonals in the order given.  The product is
 * formed exactly as written, so an Inf or NaN of x reaches y[i] through
 * every stored element of row i, zero-valued ones included.
 */
void orc_dia_spmv(int64_t N, int nd, const int64_t *offsets,
                  const int64_t *starts, const double *vals,
                  const double *x, double *y)
{
    for (int64_t i = 0; i < N; i++) {
        double ar = 0.0, ai = 0.0;
        for (int k = 0; k < nd; k++) {
            const int64_t d = offsets[k];
            const int64_t j = i + d;
            if (j < 0 || j >= N) continue;
            const int64_t t = i - (d < 0 ? -d : 0);
            const double vr = vals[2 * (starts[k] + t)];
            const double vi = vals[2 * (starts[k] + t) + 1];
            ar += vr * x[2 * j] - vi * x[2 * j + 1];
            ai += vr * x[2 * j + 1] + vi * x[2 * j];
        }
        y[2 * i] = ar;
        y[2 * i + 1] = ai;
    }
}

/* ------------------------------------------------------------------ */
/* Pauli sums                                                           */
/* ------------------------------------------------------------------ */

static int popcount64(uint64_t v)
{
    int c = 0;
    while (v) {
        v &= v - 1;
        c++;
    }
    return c;
}

/*
 * out <- H phi for H = sum_t coef[t] * P_t, P_t = i^{|x & z|} X^x Z^z.
 * On a basis state, Z^z |j> = (-1)^{|j & z|} |j> and X^x |j> = |j xor x>,
 * so (P phi)[i] = i^{|x & z|} (-1)^{|(i xor x) & z|} phi[i xor x].
 */
void orc_pauli_sum_apply(int n, int nterms, const uint64_t *xmask,
                         const uint64_t *zmask, const double *coef,
                         const double *phi, double *out)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static) if (N > 32768)
    for (int64_t i = 0; i < N; i++) {
        double ar = 0.0, ai = 0.0;
        for (int t = 0; t < nterms; t++) {
            const uint64_t j = (uint64_t)i ^ xmask[t];
            const int ny = popcount64(xmask[t] & zmask[t]) & 3;
            const int sgn = popcount64(j & zmask[t]) & 1;
            double pr = phi[2 * j], pi = phi[2 * j + 1];
            /* multiply by i^ny */
            for (int q = 0; q < ny; q++) {
                const double t0 = pr;
                pr = -pi;
                pi = t0;
            }
            if (sgn) {
                pr = -pr;
                pi = -pi;
            }
            ar += coef[t] * pr;
            ai += coef[t] * pi;
        }
        out[2 * i] = ar;
        out[2 * i + 1] = ai;
    }
}

/* One step of Neumaier's compensated summation: s + c carries the running
 * sum with its rounding error, so a 2^28-term sum stays within a few ulps
 * instead of drifting by up to N ulps. */
static void neumaier_add(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

/* <a|b> = sum_i conj(a_i) b_i, summed in index order with compensation. */
void orc_inner(int64_t N, const double *a, const double *b, double *out)
{
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    for (int64_t i = 0; i < N; i++) {
        neumaier_add(&sr, &cr, a[2 * i] * b[2 * i] + a[2 * i + 1] * b[2 * i + 1]);
        neumaier_add(&si, &ci, a[2 * i] * b[2 * i + 1] - a[2 * i + 1] * b[2 * i]);
    }
    out[0] = sr + cr;
    out[1] = si + ci;
}

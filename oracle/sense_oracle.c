/*
 * FP64 CPU oracle for multicoil Cartesian SENSE encoding and CG-SENSE.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * What it computes (plain definitions, double precision, no blocking or
 * fusion beyond what the definitions state):
 *
 *   centred unitary DFT along one axis of length N
 *       F_c v = N^(-1/2) * fftshift( DFT( ifftshift(v) ) ),
 *       DFT[k] = sum_n v[n] exp(-2 pi i k n / N)   (forward, image -> k-space)
 *       F_c^H uses exp(+2 pi i k n / N)            ("BACKWARD" direction of the
 *                                                   paper's FFT process)
 *     fftshift/ifftshift follow numpy: roll by floor(N/2) and -floor(N/2).
 *     Multi-dimensional transforms apply it axis by axis.
 *
 *   forward operator     y_c = M .* F_c( S_c .* x )                (per coil c)
 *   adjoint operator     x   = sum_c conj(S_c) .* F_c^H( M .* y_c )
 *       With M = 1 (full sampling) the adjoint is the paper's reconstruction
 *       equation (Section "Sensitivity-weighted multicoil image
 *       reconstruction", Eq. (1)): an inverse Fourier transform of every coil
 *       image, a product with the conjugate sensitivity, and a sum over coils,
 *       here with the unitary scale N^(-1/2) in place of an unscaled inverse.
 *   normal operator      A p = E^H( E p ) + lambda p   (composed, never fused)
 *   CG-SENSE             conjugate gradients on A x = E^H y from x0 = 0
 *   RSS                  sqrt( sum_c |F_c^H y_c|^2 )   (the paper's
 *                        "sum of squares" reconstruction, Section
 *                        "Performance comparison with other frameworks")
 *
 * The FFT routine is a recursive decimation-in-time mixed-radix transform
 * that splits by the smallest prime factor in {2, 3, 5} and combines with
 * p-point direct sums; anything else (and N <= 16) is a direct O(N^2) DFT.
 * Every twiddle is evaluated directly as cos/sin of 2 pi ((a b) mod N) / N.
 *
 * Layouts (x fastest, complex interleaved as numpy complex128):
 *   x    [B][Nz][Ny][Nx]
 *   maps [B or 1][C][Nz][Ny][Nx]   (maps_shared = 1: one set for all B)
 *   y    [B][C][Nz][Ny][Nx]
 *   mask [Nz][Ny] uint8 in centred order (phase-encode axes only; it
 *        broadcasts along the readout x).
 * 2D problems use ndim = 2 and Nz = 1.
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_PI 3.14159265358979323846264338327950288

/* CG stop statuses. */
enum { OR_MAXITER = 0, OR_CONVERGED = 1, OR_EXACT = 2, OR_BREAKDOWN = 3, OR_NONFINITE = 4 };

/* exp(sign * 2 pi i * e / n) with e reduced mod n first. */
static cplx twiddle(long e, long n, int sign)
{
    long r = e % n;
    if (r < 0) r += n;
    double ang = 2.0 * OR_PI * (double)r / (double)n;
    return cos(ang) + (double)sign * sin(ang) * I;
}

/* out[k] = sum_j in[j*is] exp(sign 2 pi i j k / n), for k in [0, n). */
static void dft_direct(long n, const cplx *in, ptrdiff_t is, cplx *out, int sign)
{
    for (long k = 0; k < n; ++k) {
        cplx acc = 0.0;
        for (long j = 0; j < n; ++j)
            acc += in[j * is] * twiddle(j * k, n, sign);
        out[k] = acc;
    }
}

static long smallest_factor235(long n)
{
    if (n % 2 == 0) return 2;
    if (n % 3 == 0) return 3;
    if (n % 5 == 0) return 5;
    return 0;
}

/*
 * Decimation in time: with n = p m, x[p j + r] for r in [0, p) are p
 * sequences of length m with DFTs Y_r.  Then
 *     X[k] = sum_r exp(sign 2 pi i r k / n) Y_r[k mod m],  k in [0, n).
 */
static void fft_rec(long n, const cplx *in, ptrdiff_t is, cplx *out, int sign)
{
    long p = smallest_factor235(n);
    if (n <= 16 || p == 0) {
        dft_direct(n, in, is, out, sign);
        return;
    }
    long m = n / p;
    cplx *sub = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (long r = 0; r < p; ++r)
        fft_rec(m, in + r * is, is * p, sub + r * m, sign);
    for (long k = 0; k < n; ++k) {
        cplx acc = 0.0;
        for (long r = 0; r < p; ++r)
            acc += sub[r * m + (k % m)] * twiddle(r * k, n, sign);
        out[k] = acc;
    }
    free(sub);
}

/* Unnormalised DFT of length n (sign -1 forward, +1 inverse). */
int or_fft1d(long n, const cplx *in, cplx *out, int sign)
{
    if (n <= 0 || (sign != 1 && sign != -1)) return -1;
    fft_rec(n, in, 1, out, sign);
    return 0;
}

/* Direct O(n^2) DFT, exposed so tests can compare it with the FFT routine. */
int or_dft1d_direct(long n, const cplx *in, cplx *out, int sign)
{
    if (n <= 0 || (sign != 1 && sign != -1)) return -1;
    dft_direct(n, in, 1, out, sign);
    return 0;
}

/*
 * Centred unitary transform of one line (length n, element stride s), in
 * place.  dir = -1: F_c, dir = +1: F_c^H.
 *   ifftshift: t[i] = v[(i + n/2) mod n]      (roll by -floor(n/2))
 *   DFT
 *   fftshift:  v[i] = T[(i - n/2) mod n]      (roll by +floor(n/2))
 *   scale by n^(-1/2)
 */
static void centred_line(long n, cplx *v, ptrdiff_t s, int dir, cplx *t, cplx *T)
{
    long h = n / 2;
    for (long i = 0; i < n; ++i) t[i] = v[((i + h) % n) * s];
    fft_rec(n, t, 1, T, dir);
    double sc = 1.0 / sqrt((double)n);
    for (long i = 0; i < n; ++i) v[i * s] = T[((i - h) % n + n) % n] * sc;
}

int or_centred1d(long n, const cplx *in, cplx *out, int dir)
{
    if (n <= 0 || (dir != 1 && dir != -1)) return -1;
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)n * 2);
    memcpy(out, in, sizeof(cplx) * (size_t)n);
    centred_line(n, out, 1, dir, t, t + n);
    free(t);
    return 0;
}

/* Centred unitary multi-dimensional transform of one [nz][ny][nx] image in
 * place: along x, then y, then z (each axis of length > 1). */
static void centred_nd(cplx *img, long nx, long ny, long nz, int dir)
{
    long nmax = nx > ny ? nx : ny;
    if (nz > nmax) nmax = nz;
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)nmax * 2);
    if (nx > 1)
        for (long z = 0; z < nz; ++z)
            for (long y = 0; y < ny; ++y)
                centred_line(nx, img + (z * ny + y) * nx, 1, dir, t, t + nmax);
    if (ny > 1)
        for (long z = 0; z < nz; ++z)
            for (long x = 0; x < nx; ++x)
                centred_line(ny, img + z * ny * nx + x, nx, dir, t, t + nmax);
    if (nz > 1)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x)
                centred_line(nz, img + y * nx + x, nx * ny, dir, t, t + nmax);
    free(t);
}

int or_centred_nd(const cplx *in, cplx *out, long nx, long ny, long nz, int dir)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || (dir != 1 && dir != -1)) return -1;
    memcpy(out, in, sizeof(cplx) * (size_t)(nx * ny * nz));
    centred_nd(out, nx, ny, nz, dir);
    return 0;
}

/* Mask value at voxel (z, y, x): the phase-encode mask broadcasts along x. */
static double mask_at(const uint8_t *mask, long ny, long z, long y)
{
    return mask[z * ny + y] ? 1.0 : 0.0;
}

static int check_dims(long nx, long ny, long nz, int ncoils, int batch)
{
    return (nx > 0 && ny > 0 && nz > 0 && ncoils > 0 && batch > 0) ? 0 : -1;
}

/* Forward operator: y[b][c] = M .* F_c(S[b][c] .* x[b]). */
int or_E(long nx, long ny, long nz, int ncoils, int batch, int maps_shared,
         const cplx *x, const cplx *maps, const uint8_t *mask, cplx *y)
{
    if (check_dims(nx, ny, nz, ncoils, batch)) return -1;
    long nvox = nx * ny * nz;
    long jobs = (long)batch * ncoils;
#pragma omp parallel for schedule(dynamic, 1)
    for (long j = 0; j < jobs; ++j) {
        long b = j / ncoils, c = j % ncoils;
        const cplx *s = maps + ((maps_shared ? 0 : b) * ncoils + c) * nvox;
        const cplx *xb = x + b * nvox;
        cplx *yc = y + (b * ncoils + c) * nvox;
        for (long v = 0; v < nvox; ++v) yc[v] = s[v] * xb[v];
        centred_nd(yc, nx, ny, nz, -1);
        for (long z = 0; z < nz; ++z)
            for (long yy = 0; yy < ny; ++yy) {
                double m = mask_at(mask, ny, z, yy);
                for (long xx = 0; xx < nx; ++xx) yc[(z * ny + yy) * nx + xx] *= m;
            }
    }
    return 0;
}

/* Adjoint operator: x[b] = sum_c conj(S[b][c]) .* F_c^H(M .* y[b][c]),
 * coils summed in increasing c. */
int or_EH(long nx, long ny, long nz, int ncoils, int batch, int maps_shared,
          const cplx *y, const cplx *maps, const uint8_t *mask, cplx *x)
{
    if (check_dims(nx, ny, nz, ncoils, batch)) return -1;
    long nvox = nx * ny * nz;
    long jobs = (long)batch * ncoils;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)(jobs * nvox));
    if (!tmp) return -2;
#pragma omp parallel for schedule(dynamic, 1)
    for (long j = 0; j < jobs; ++j) {
        long b = j / ncoils, c = j % ncoils;
        const cplx *s = maps + ((maps_shared ? 0 : b) * ncoils + c) * nvox;
        const cplx *yc = y + j * nvox;
        cplx *t = tmp + j * nvox;
        for (long z = 0; z < nz; ++z)
            for (long yy = 0; yy < ny; ++yy) {
                double m = mask_at(mask, ny, z, yy);
                for (long xx = 0; xx < nx; ++xx) {
                    long v = (z * ny + yy) * nx + xx;
                    t[v] = yc[v] * m;
                }
            }
        centred_nd(t, nx, ny, nz, +1);
        for (long v = 0; v < nvox; ++v) t[v] = conj(s[v]) * t[v];
    }
    for (long b = 0; b < batch; ++b) {
        cplx *xb = x + b * nvox;
        for (long v = 0; v < nvox; ++v) {
            cplx acc = 0.0;
            for (long c = 0; c < ncoils; ++c) acc += tmp[(b * ncoils + c) * nvox + v];
            xb[v] = acc;
        }
    }
    free(tmp);
    return 0;
}

/* Normal operator, composed: q = E^H(E p) + lambda p. */
int or_A(long nx, long ny, long nz, int ncoils, int batch, int maps_shared,
         const cplx *p, const cplx *maps, const uint8_t *mask, double lambda, cplx *q)
{
    if (check_dims(nx, ny, nz, ncoils, batch)) return -1;
    long nvox = nx * ny * nz;
    cplx *k = (cplx *)malloc(sizeof(cplx) * (size_t)((long)batch * ncoils * nvox));
    if (!k) return -2;
    int rc = or_E(nx, ny, nz, ncoils, batch, maps_shared, p, maps, mask, k);
    if (!rc) rc = or_EH(nx, ny, nz, ncoils, batch, maps_shared, k, maps, mask, q);
    free(k);
    if (rc) return rc;
    for (long v = 0; v < (long)batch * nvox; ++v) q[v] += lambda * p[v];
    return 0;
}

/* <a, b> = sum conj(a) b */
static cplx dotc(const cplx *a, const cplx *b, long n)
{
    cplx acc = 0.0;
    for (long i = 0; i < n; ++i) acc += conj(a[i]) * b[i];
    return acc;
}

/*
 * CG-SENSE: conjugate gradients on the normal equations A x = b, b = E^H y,
 * independently for every batch element.
 *
 *   x = 0, r = b, p = r, rho = <r, r>, rho0 = rho
 *   for k = 0 .. max_iter-1:
 *       rho == 0                    -> EXACT
 *       q = A p, eta = Re <p, q>
 *       eta not finite              -> NONFINITE;  eta <= 0 -> BREAKDOWN
 *       alpha = rho / eta
 *       x += alpha p;  r -= alpha q;  rho' = <r, r>
 *       rho' not finite             -> NONFINITE
 *       tol > 0 and sqrt(rho'/rho0) < tol -> CONVERGED
 *       beta = rho' / rho;  p = r + beta p;  rho = rho'
 *   otherwise                       -> MAXITER
 *
 * rho_hist (per batch element, max_iter + 1 entries) receives rho0 and each
 * rho'; iters[b] the number of completed updates of x; status[b] the reason
 * the loop ended.
 *
 * vec32 != 0 stores every CG vector in single precision: b = E^H y, each
 * q = A p and each new x, r and p are rounded to binary32 components as they
 * are produced, while the operator, the inner products and alpha, beta stay
 * in double.  This is the same loop with complex64 storage and exact
 * arithmetic otherwise: the floor that complex64 storage alone puts under
 * any fp32 implementation of the solve.
 */
/* Round both components to the nearest binary32 value (ties to even). */
static cplx round32(cplx v)
{
    return (double)(float)creal(v) + I * (double)(float)cimag(v);
}

static void round32_vec(cplx *v, long n, int on)
{
    if (!on) return;
    for (long i = 0; i < n; ++i) v[i] = round32(v[i]);
}

int or_cg(long nx, long ny, long nz, int ncoils, int batch, int maps_shared,
          const cplx *y, const cplx *maps, const uint8_t *mask,
          int max_iter, double tol, double lambda, int vec32,
          cplx *x, int *iters, int *status, double *rho_hist)
{
    if (check_dims(nx, ny, nz, ncoils, batch) || max_iter < 0) return -1;
    long nvox = nx * ny * nz;
    for (int b = 0; b < batch; ++b) {
        const cplx *yb = y + (long)b * ncoils * nvox;
        const cplx *sb = maps + (maps_shared ? 0 : (long)b * ncoils * nvox);
        cplx *xb = x + (long)b * nvox;
        double *hist = rho_hist + (long)b * (max_iter + 1);
        cplx *r = (cplx *)malloc(sizeof(cplx) * (size_t)nvox * 3);
        if (!r) return -2;
        cplx *p = r + nvox, *q = r + 2 * nvox;
        for (int k = 0; k <= max_iter; ++k) hist[k] = 0.0;

        int rc = or_EH(nx, ny, nz, ncoils, 1, 1, yb, sb, mask, r);
        if (rc) { free(r); return rc; }
        round32_vec(r, nvox, vec32);
        for (long v = 0; v < nvox; ++v) { xb[v] = 0.0; p[v] = r[v]; }
        double rho = creal(dotc(r, r, nvox)), rho0 = rho;
        hist[0] = rho;
        int st = OR_MAXITER, k = 0;
        if (!isfinite(rho)) st = OR_NONFINITE;
        for (; st == OR_MAXITER && k < max_iter;) {
            if (rho == 0.0) { st = OR_EXACT; break; }
            rc = or_A(nx, ny, nz, ncoils, 1, 1, p, sb, mask, lambda, q);
            if (rc) { free(r); return rc; }
            round32_vec(q, nvox, vec32);
            double eta = creal(dotc(p, q, nvox));
            if (!isfinite(eta)) { st = OR_NONFINITE; break; }
            if (eta <= 0.0) { st = OR_BREAKDOWN; break; }
            double alpha = rho / eta;
            for (long v = 0; v < nvox; ++v) {
                xb[v] += alpha * p[v];
                r[v] -= alpha * q[v];
            }
            round32_vec(xb, nvox, vec32);
            round32_vec(r, nvox, vec32);
            double rho_new = creal(dotc(r, r, nvox));
            ++k;
            hist[k] = rho_new;
            if (!isfinite(rho_new)) { st = OR_NONFINITE; break; }
            if (tol > 0.0 && sqrt(rho_new / rho0) < tol) { st = OR_CONVERGED; break; }
            double beta = rho_new / rho;
            for (long v = 0; v < nvox; ++v) p[v] = r[v] + beta * p[v];
            round32_vec(p, nvox, vec32);
            rho = rho_new;
        }
        iters[b] = k;
        status[b] = st;
        free(r);
    }
    return 0;
}

/* Threads of the calling thread's later parallel regions (timing only; the
 * results do not depend on it).  Returns the threads now in effect. */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Root sum of squares: out[b] = sqrt( sum_c |F_c^H y[b][c]|^2 ), no mask. */
int or_rss(long nx, long ny, long nz, int ncoils, int batch, const cplx *y, double *out)
{
    if (check_dims(nx, ny, nz, ncoils, batch)) return -1;
    long nvox = nx * ny * nz;
    long jobs = (long)batch * ncoils;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)(jobs * nvox));
    if (!tmp) return -2;
#pragma omp parallel for schedule(dynamic, 1)
    for (long j = 0; j < jobs; ++j) {
        memcpy(tmp + j * nvox, y + j * nvox, sizeof(cplx) * (size_t)nvox);
        centred_nd(tmp + j * nvox, nx, ny, nz, +1);
    }
    for (long b = 0; b < batch; ++b)
        for (long v = 0; v < nvox; ++v) {
            double acc = 0.0;
            for (long c = 0; c < ncoils; ++c) {
                cplx t = tmp[(b * ncoils + c) * nvox + v];
                acc += creal(t) * creal(t) + cimag(t) * cimag(t);
            }
            out[b * nvox + v] = sqrt(acc);
        }
    free(tmp);
    return 0;
}

/*
 * FP64 CPU oracle for free-space propagation of sampled optical fields.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (TorchOptics paper, section "Computational Fourier
 * optics"):
 *   - the angular-spectrum (AS) propagation of Eq. (field_propagation_tf)
 *     with the transfer function of Eq. (transfer_function), evaluated on a
 *     zero-padded grid with the discrete Fourier transform;
 *   - the Fresnel transfer-function variant of the same pipeline;
 *   - the direct-integration (DI) method: Eq. (field_propagation) as a
 *     discrete linear convolution with the sampled impulse response of
 *     Eq. (impulse_response), computed with the same zero-padded DFT
 *     pipeline (the transfer function is the DFT of the sampled response);
 *   - the adjoint of that linear operator;
 *   - a brute-force Rayleigh-Sommerfeld sum of Eq. (field_propagation) with
 *     the impulse response of Eq. (impulse_response), used as a physics
 *     cross-check.
 *
 * Everything is double precision; transfer-function and twiddle phases are
 * evaluated in long double (x86-64 80-bit) and reduced modulo one cycle
 * before the exponential.  The FFT is a plain iterative radix-2 transform
 * with its own twiddle table (no recurrences); a naive O(n^2) DFT is provided
 * as an independent check of it.
 *
 * Complex arrays are C99 double _Complex, which has the memory layout of
 * numpy complex128 (interleaved re, im).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

#define ORC_ASM 0
#define ORC_FRESNEL 1
#define ORC_DI 2

static const long double TWO_PI_L = 6.283185307179586476925286766559005768L;

/* exp(2*pi*i*c) for a phase c given in cycles; c is first reduced to [0,1). */
static cplx cis_cycles(long double c)
{
    long double fr = c - floorl(c);
    long double a = TWO_PI_L * fr;
    return (double)cosl(a) + I * (double)sinl(a);
}

/* ---------------------------------------------------------------------- */
/* Discrete Fourier transform                                              */
/* ---------------------------------------------------------------------- */

/* Naive DFT: y[k] = sum_n x[n] exp(sign * 2 pi i n k / n_len).  The product
 * n*k is reduced modulo n_len in integers, so the angle is exact before the
 * long-double sine/cosine. */
void orc_dft(const cplx *x, cplx *y, long n, int sign)
{
    for (long k = 0; k < n; ++k) {
        long double sr = 0.0L, si = 0.0L;
        for (long j = 0; j < n; ++j) {
            long m = (long)(((unsigned long)j * (unsigned long)k) % (unsigned long)n);
            long double a = (long double)sign * TWO_PI_L * (long double)m / (long double)n;
            long double c = cosl(a), s = sinl(a);
            long double xr = creal(x[j]), xi = cimag(x[j]);
            sr += xr * c - xi * s;
            si += xr * s + xi * c;
        }
        y[k] = (double)sr + I * (double)si;
    }
}

static int is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

/* In-place iterative radix-2 FFT (decimation in time), unnormalised:
 * x[k] <- sum_n x[n] exp(sign * 2 pi i n k / n).  Returns -1 if n is not a
 * power of two. */
int orc_fft(cplx *x, long n, int sign)
{
    if (!is_pow2(n)) return -1;
    if (n == 1) return 0;
    /* bit-reversal permutation */
    for (long i = 1, j = 0; i < n; ++i) {
        long bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    /* twiddles w[m] = exp(sign * 2 pi i m / n), m < n/2, each from its own
     * long-double sine/cosine */
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)(n / 2));
    for (long m = 0; m < n / 2; ++m) {
        long double a = (long double)sign * TWO_PI_L * (long double)m / (long double)n;
        w[m] = (double)cosl(a) + I * (double)sinl(a);
    }
    for (long len = 2; len <= n; len <<= 1) {
        long half = len >> 1, step = n / len;
        for (long s = 0; s < n; s += len) {
            for (long k = 0; k < half; ++k) {
                cplx t = w[k * step] * x[s + k + half];
                cplx u = x[s + k];
                x[s + k] = u + t;
                x[s + k + half] = u - t;
            }
        }
    }
    free(w);
    return 0;
}

/* 2-D FFT of a row-major ny x nx array (x fastest): rows, then columns. */
int orc_fft2(cplx *a, long ny, long nx, int sign)
{
    if (!is_pow2(ny) || !is_pow2(nx)) return -1;
    for (long r = 0; r < ny; ++r) orc_fft(a + r * nx, nx, sign);
    cplx *col = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
    for (long c = 0; c < nx; ++c) {
        for (long r = 0; r < ny; ++r) col[r] = a[r * nx + c];
        orc_fft(col, ny, sign);
        for (long r = 0; r < ny; ++r) a[r * nx + c] = col[r];
    }
    free(col);
    return 0;
}

/* In-place 1-D transform of any length: the radix-2 FFT for powers of two,
 * the naive DFT (integer-reduced long-double angles) otherwise. */
static void dft_any(cplx *x, long n, int sign, cplx *tmp)
{
    if (is_pow2(n)) {
        orc_fft(x, n, sign);
        return;
    }
    orc_dft(x, tmp, n, sign);
    memcpy(x, tmp, sizeof(cplx) * (size_t)n);
}

/* 2-D transform of a row-major ny x nx array of any extents (rows, then
 * columns).  Non-power-of-two extents take O(n^2) per line: small grids. */
int orc_dft2_any(cplx *a, long ny, long nx, int sign)
{
    if (ny < 1 || nx < 1) return -1;
    long m = ny > nx ? ny : nx;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)m);
    cplx *col = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
    for (long r = 0; r < ny; ++r) dft_any(a + r * nx, nx, sign, tmp);
    for (long c = 0; c < nx; ++c) {
        for (long r = 0; r < ny; ++r) col[r] = a[r * nx + c];
        dft_any(col, ny, sign, tmp);
        for (long r = 0; r < ny; ++r) a[r * nx + c] = col[r];
    }
    free(col);
    free(tmp);
    return 0;
}

/* The same 2-D transform with its lines shared among the threads of the
 * enclosing OpenMP team (call from inside a parallel region, by every
 * thread): each row and each column is transformed exactly as above, only
 * by whichever thread takes it.  Used when a call has fewer fields than
 * threads, so that one large field still occupies every core. */
static void dft2_any_team(cplx *a, long ny, long nx, int sign)
{
    long m = ny > nx ? ny : nx;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)m);
    cplx *col = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
#pragma omp for schedule(static)
    for (long r = 0; r < ny; ++r) dft_any(a + r * nx, nx, sign, tmp);
#pragma omp for schedule(static)
    for (long c = 0; c < nx; ++c) {
        for (long r = 0; r < ny; ++r) col[r] = a[r * nx + c];
        dft_any(col, ny, sign, tmp);
        for (long r = 0; r < ny; ++r) a[r * nx + c] = col[r];
    }
    free(col);
    free(tmp);
}

/* ---------------------------------------------------------------------- */
/* Transfer functions                                                      */
/* ---------------------------------------------------------------------- */

/* Spatial frequency of DFT bin k on a length-n grid of spacing d, in cycles
 * per metre, with numpy's fftfreq ordering (bins with 2k >= n are negative,
 * which for odd n keeps bin (n-1)/2 positive). */
static long double freq_of_bin(long k, long n, double d)
{
    long ks = (2 * k < n) ? k : k - n;
    return (long double)ks / ((long double)n * (long double)d);
}

/* Phase, in cycles, of the transfer function at spatial frequency (fx, fy).
 *
 * AS method, Eq. (transfer_function): H = exp(i z sqrt(k^2 - kx^2 - ky^2))
 * with k = 2 pi / lambda and kx = 2 pi fx, i.e. a phase of
 * z * sqrt(1/lambda^2 - fx^2 - fy^2) cycles.  The paper does not say what is
 * done where the root is imaginary; this oracle zeroes those (evanescent)
 * components, keeping the boundary where the root is exactly zero.
 *
 * Fresnel transfer function (the paraxial approximation the paper offers as
 * an alternative): phase z/lambda - (lambda z / 2)(fx^2 + fy^2) cycles.
 *
 * Returns 0 and sets *valid = 0 for an evanescent AS component. */
static long double tf_phase_cycles(long double fx, long double fy, double lam, double z,
                                   int method, int *valid)
{
    long double L = (long double)lam, Z = (long double)z;
    long double rho2 = fx * fx + fy * fy;
    *valid = 1;
    if (method == ORC_FRESNEL)
        return Z / L - 0.5L * L * Z * rho2;
    long double arg = 1.0L / (L * L) - rho2;
    if (arg < 0.0L) { *valid = 0; return 0.0L; }
    return Z * sqrtl(arg);
}

/* Transfer function on a py x px grid of DFT bins (row-major, FFT order). */
void orc_transfer(cplx *H, long py, long px, double dy, double dx, double lam, double z,
                  int method)
{
#pragma omp parallel for schedule(static)
    for (long ky = 0; ky < py; ++ky) {
        long double fy = freq_of_bin(ky, py, dy);
        for (long kx = 0; kx < px; ++kx) {
            long double fx = freq_of_bin(kx, px, dx);
            int valid;
            long double c = tf_phase_cycles(fx, fy, lam, z, method, &valid);
            H[ky * px + kx] = valid ? cis_cycles(c) : 0.0;
        }
    }
}

/* Impulse response of Eq. (impulse_response) at lateral offset (ox, oy):
 *   h = z / (i lambda d) * (1 + i / (k d)) * exp(i k d) / d,
 *   d = sqrt(ox^2 + oy^2 + z^2),  k = 2 pi / lambda,
 * with the phase k d carried as d / lambda cycles in long double. */
static cplx impulse_response(long double oy, long double ox, double lam, double z)
{
    long double L = (long double)lam, Z = (long double)z;
    long double d = sqrtl(ox * ox + oy * oy + Z * Z);
    long double kd = TWO_PI_L * d / L;
    cplx pre = (double)(Z / (L * d * d)) / I;
    cplx corr = 1.0 + I * (double)(1.0L / kd);
    return pre * corr * cis_cycles(d / L);
}

/* Transfer function of the DI method on a py x px grid (FFT order): the
 * forward DFT of the impulse response sampled at the lateral offsets the
 * discrete convolution of an ny x nx field with itself can produce, times
 * the area element dx dy of the Riemann sum of Eq. (field_propagation).
 * Entry (ky, kx) of the sampled response holds the offset (sy dy, sx dx)
 * with sy = ky (ky < py/2) or ky - py (signed, as the circular index of a
 * difference of two positions); offsets with |sy| >= ny or |sx| >= nx can
 * never occur between two samples of the field and are zero.  With
 * py >= 2 ny - 1 and px >= 2 nx - 1 the circular convolution of the
 * zero-padded field with this array equals the linear one on the kept
 * window.  Returns -1 when the padding is too small for that. */
int orc_di_transfer(cplx *H, long ny, long nx, long py, long px, double dy, double dx, double lam,
                    double z)
{
    if (py < 2 * ny - 1 || px < 2 * nx - 1) return -1;
    for (long ky = 0; ky < py; ++ky) {
        long sy = (2 * ky < py) ? ky : ky - py;
        for (long kx = 0; kx < px; ++kx) {
            long sx = (2 * kx < px) ? kx : kx - px;
            if (labs(sy) >= ny || labs(sx) >= nx) {
                H[ky * px + kx] = 0.0;
                continue;
            }
            H[ky * px + kx] = impulse_response((long double)sy * dy, (long double)sx * dx, lam, z) * dx * dy;
        }
    }
    return orc_dft2_any(H, py, px, -1);
}

/* Transfer function of `method` for an ny x nx field on a py x px grid. */
static int method_transfer(cplx *H, long ny, long nx, long py, long px, double dy, double dx,
                           double lam, double z, int method)
{
    if (method == ORC_DI) return orc_di_transfer(H, ny, nx, py, px, dy, dx, lam, z);
    if (method != ORC_ASM && method != ORC_FRESNEL) return -1;
    orc_transfer(H, py, px, dy, dx, lam, z, method);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Propagation                                                             */
/* ---------------------------------------------------------------------- */

/* One propagation of an ny x nx field through distance z (section
 * "Computational Fourier optics", Eq. (field_propagation_tf)):
 *   1. zero-pad to py x px (py >= ny, px >= nx), the field centred in a window
 *      starting at ((py-ny)/2, (px-nx)/2) (integer division);
 *   2. forward 2-D DFT;
 *   3. multiply by the transfer function H (or by conj(H) when adjoint != 0,
 *      which is the Hermitian adjoint of the whole operator because the
 *      crop is the adjoint of the pad and the unnormalised DFT pair is
 *      unitary up to the 1/(py*px) factor);
 *   4. inverse 2-D DFT scaled by 1/(py*px);
 *   5. crop the same window.
 * H is passed in (from orc_transfer or orc_di_transfer) so a batch shares
 * one table. */
static void propagate_one(const cplx *in, cplx *out, cplx *work, const cplx *H, long ny,
                          long nx, long py, long px, int adjoint)
{
    long oy = (py - ny) / 2, ox = (px - nx) / 2;
    memset(work, 0, sizeof(cplx) * (size_t)(py * px));
    for (long r = 0; r < ny; ++r)
        memcpy(work + (r + oy) * px + ox, in + r * nx, sizeof(cplx) * (size_t)nx);
    orc_dft2_any(work, py, px, -1);
    for (long i = 0; i < py * px; ++i) work[i] *= adjoint ? conj(H[i]) : H[i];
    orc_dft2_any(work, py, px, +1);
    double scale = 1.0 / ((double)py * (double)px);
    for (long r = 0; r < ny; ++r)
        for (long c = 0; c < nx; ++c) out[r * nx + c] = work[(r + oy) * px + c + ox] * scale;
}

/* propagate_one with every step shared among the threads of the enclosing
 * team (call from inside a parallel region, by every thread); `work` is
 * shared.  Same arithmetic per element and per line as propagate_one. */
static void propagate_one_team(const cplx *in, cplx *out, cplx *work, const cplx *H, long ny,
                               long nx, long py, long px, int adjoint)
{
    long oy = (py - ny) / 2, ox = (px - nx) / 2;
#pragma omp for schedule(static)
    for (long r = 0; r < py; ++r) {
        memset(work + r * px, 0, sizeof(cplx) * (size_t)px);
        if (r >= oy && r < oy + ny)
            memcpy(work + r * px + ox, in + (r - oy) * nx, sizeof(cplx) * (size_t)nx);
    }
    dft2_any_team(work, py, px, -1);
#pragma omp for schedule(static)
    for (long i = 0; i < py * px; ++i) work[i] *= adjoint ? conj(H[i]) : H[i];
    dft2_any_team(work, py, px, +1);
    double scale = 1.0 / ((double)py * (double)px);
#pragma omp for schedule(static)
    for (long r = 0; r < ny; ++r)
        for (long c = 0; c < nx; ++c) out[r * nx + c] = work[(r + oy) * px + c + ox] * scale;
}

/* Batched propagation of `batch` contiguous ny x nx fields on a py x px
 * padded grid.  Returns -1 for an unsupported size (padded extents no
 * smaller than the field; extents that are not powers of two use the naive
 * DFT, so they are meant for small grids). */
int orc_propagate(const cplx *in, cplx *out, long batch, long ny, long nx, long py, long px,
                  double dy, double dx, double lam, double z, int method, int adjoint)
{
    if (ny < 1 || nx < 1 || py < ny || px < nx) return -1;
    cplx *H = (cplx *)malloc(sizeof(cplx) * (size_t)(py * px));
    if (method_transfer(H, ny, nx, py, px, dy, dx, lam, z, method) != 0) {
        free(H);
        return -1;
    }
    if (batch >= omp_get_max_threads()) {
        /* one field per thread at a time */
#pragma omp parallel
        {
            cplx *work = (cplx *)malloc(sizeof(cplx) * (size_t)(py * px));
#pragma omp for schedule(dynamic, 1)
            for (long b = 0; b < batch; ++b)
                propagate_one(in + b * ny * nx, out + b * ny * nx, work, H, ny, nx, py, px, adjoint);
            free(work);
        }
    } else {
        /* fewer fields than threads: the threads share each field's lines */
        cplx *work = (cplx *)malloc(sizeof(cplx) * (size_t)(py * px));
#pragma omp parallel
        for (long b = 0; b < batch; ++b)
            propagate_one_team(in + b * ny * nx, out + b * ny * nx, work, H, ny, nx, py, px, adjoint);
        free(work);
    }
    free(H);
    return 0;
}

/* Same operator, but with the field placed at an arbitrary window offset
 * (oy, ox) inside the padded grid.  Used only to test that the result does
 * not depend on where the zero padding goes. */
int orc_propagate_offset(const cplx *in, cplx *out, long ny, long nx, long py, long px, long oy,
                         long ox, double dy, double dx, double lam, double z, int method)
{
    if (oy < 0 || ox < 0 || oy + ny > py || ox + nx > px) return -1;
    cplx *H = (cplx *)malloc(sizeof(cplx) * (size_t)(py * px));
    cplx *work = (cplx *)calloc((size_t)(py * px), sizeof(cplx));
    if (method_transfer(H, ny, nx, py, px, dy, dx, lam, z, method) != 0) {
        free(work);
        free(H);
        return -1;
    }
    for (long r = 0; r < ny; ++r)
        memcpy(work + (r + oy) * px + ox, in + r * nx, sizeof(cplx) * (size_t)nx);
    orc_dft2_any(work, py, px, -1);
    for (long i = 0; i < py * px; ++i) work[i] *= H[i];
    orc_dft2_any(work, py, px, +1);
    double scale = 1.0 / ((double)py * (double)px);
    for (long r = 0; r < ny; ++r)
        for (long c = 0; c < nx; ++c) out[r * nx + c] = work[(r + oy) * px + c + ox] * scale;
    free(work);
    free(H);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Rayleigh-Sommerfeld brute force                                         */
/* ---------------------------------------------------------------------- */

/* Direct Riemann sum of Eq. (field_propagation) with the impulse response of
 * Eq. (impulse_response):
 *   h = z / (i lambda d) * (1 + i / (k d)) * exp(i k d) / d,
 *   d = sqrt((x - x')^2 + (y - y')^2 + z^2),  k = 2 pi / lambda,
 * on the same grid for input and output (spacing dy, dx), weighted by the
 * area element dx*dy.  O(N^4): for tiny grids only. */
void orc_rs_direct(const cplx *in, cplx *out, long ny, long nx, double dy, double dx, double lam,
                   double z)
{
    long double k = TWO_PI_L / (long double)lam;
#pragma omp parallel for collapse(2)
    for (long r = 0; r < ny; ++r) {
        for (long c = 0; c < nx; ++c) {
            cplx acc = 0.0;
            for (long rp = 0; rp < ny; ++rp) {
                for (long cp = 0; cp < nx; ++cp) {
                    long double ddy = (long double)(r - rp) * dy;
                    long double ddx = (long double)(c - cp) * dx;
                    long double d = sqrtl(ddx * ddx + ddy * ddy + (long double)z * z);
                    /* exp(i k d) with the phase k d / (2 pi) = d / lambda cycles */
                    cplx e = cis_cycles(d / (long double)lam);
                    cplx pre = (double)((long double)z / ((long double)lam * d * d)) / I;
                    cplx corr = 1.0 + I * (double)(1.0L / (k * d));
                    acc += pre * corr * e * in[rp * nx + cp];
                }
            }
            out[r * nx + c] = acc * dx * dy;
        }
    }
}

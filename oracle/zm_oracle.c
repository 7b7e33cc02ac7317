/*
 * zm_oracle.c -- plain, slow FP64 CPU oracle for Zernike moments.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes (Al-Rawi, "Ultra-Fast Zernike Moments using FFT and GPU"):
 *   - zmo_zrp_column / zmo_zrp_table: the radial polynomial R_nm of eq. (2),
 *     Sec. 2, evaluated EXACTLY in big-integer arithmetic at a point whose
 *     squared radius is a rational a/b, then rounded once (through an 80-bit
 *     long double, relative error < 2^-61 before the final rounding) to FP64.
 *     The factorial series is ill-conditioned (its terms reach ~2^(1.25 n)),
 *     so exact arithmetic is the only plain way to make it an oracle.
 *   - zmo_resample: the polar image f^(rho, theta) needed by eq. (1), by
 *     bilinear interpolation of the pixel grid (Sec. 2.5), FP64.
 *   - zmo_angular_dft: the inner angular sum of eq. (1) on a uniform grid,
 *     G[r][m] = sum_a f^[r][a] exp(-j m theta_a), written out as a plain DFT.
 *   - zmo_radial_sum: the outer radial sum of eq. (1), with the (n+1)/pi
 *     factor, the ring weights rho_r drho and the optional Neumann factor of
 *     eq. (14)-(15).
 *   - zmo_cartesian: the Cartesian pixel sum of eq. (3) with the first-order
 *     kernel of eq. (5) (a sanity check, not a parity reference).
 *   - zmo_reconstruct: the image series of eq. (9) at given points.
 *
 * Everything is FP64 (plus exact integers); loops run in a fixed order so
 * each output is a deterministic function of the inputs.  OpenMP only
 * distributes independent outputs over threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Unsigned big integers: little-endian 64-bit limbs, heap storage.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int len;       /* limbs in use; 0 means the value 0 */
    int cap;
    uint64_t* d;
} big;

static void big_init(big* x, int cap) {
    x->len = 0;
    x->cap = cap < 4 ? 4 : cap;
    x->d = (uint64_t*)calloc((size_t)x->cap, sizeof(uint64_t));
}
static void big_free(big* x) { free(x->d); x->d = NULL; x->len = x->cap = 0; }
static void big_reserve(big* x, int cap) {
    if (cap <= x->cap) return;
    x->d = (uint64_t*)realloc(x->d, (size_t)cap * sizeof(uint64_t));
    memset(x->d + x->cap, 0, (size_t)(cap - x->cap) * sizeof(uint64_t));
    x->cap = cap;
}
static void big_trim(big* x) { while (x->len > 0 && x->d[x->len - 1] == 0) x->len--; }
static void big_set_u64(big* x, uint64_t v) {
    x->len = 0;
    if (v) { x->d[0] = v; x->len = 1; }
}
static void big_copy(big* dst, const big* src) {
    big_reserve(dst, src->len + 1);
    memcpy(dst->d, src->d, (size_t)src->len * sizeof(uint64_t));
    dst->len = src->len;
}
/* x *= v */
static void big_mul_u64(big* x, uint64_t v) {
    if (x->len == 0) return;
    if (v == 0) { x->len = 0; return; }
    big_reserve(x, x->len + 1);
    unsigned __int128 carry = 0;
    for (int i = 0; i < x->len; ++i) {
        unsigned __int128 t = (unsigned __int128)x->d[i] * v + carry;
        x->d[i] = (uint64_t)t;
        carry = t >> 64;
    }
    if (carry) x->d[x->len++] = (uint64_t)carry;
}
/* x <<= s */
static void big_shl(big* x, int s) {
    if (x->len == 0 || s == 0) return;
    int w = s / 64, b = s % 64;
    big_reserve(x, x->len + w + 1);
    x->d[x->len + w] = 0;
    if (b == 0) {
        for (int i = x->len - 1; i >= 0; --i) x->d[i + w] = x->d[i];
    } else {
        for (int i = x->len - 1; i >= 0; --i) {
            x->d[i + w + 1] |= x->d[i] >> (64 - b);
            x->d[i + w] = x->d[i] << b;
        }
    }
    for (int i = 0; i < w; ++i) x->d[i] = 0;
    x->len += w + 1;
    big_trim(x);
}
/* out = x * y (schoolbook); out must not alias x or y */
static void big_mul(big* out, const big* x, const big* y) {
    if (x->len == 0 || y->len == 0) { out->len = 0; return; }
    int n = x->len + y->len;
    big_reserve(out, n);
    memset(out->d, 0, (size_t)n * sizeof(uint64_t));
    for (int i = 0; i < x->len; ++i) {
        unsigned __int128 carry = 0;
        for (int j = 0; j < y->len; ++j) {
            unsigned __int128 t = (unsigned __int128)x->d[i] * y->d[j] + out->d[i + j] + carry;
            out->d[i + j] = (uint64_t)t;
            carry = t >> 64;
        }
        int k = i + y->len;
        while (carry) {
            unsigned __int128 t = (unsigned __int128)out->d[k] + carry;
            out->d[k] = (uint64_t)t;
            carry = t >> 64;
            ++k;
        }
    }
    out->len = n;
    big_trim(out);
}
/* x += y */
static void big_add(big* x, const big* y) {
    int n = x->len > y->len ? x->len : y->len;
    big_reserve(x, n + 1);
    for (int i = x->len; i < n + 1; ++i) x->d[i] = 0;
    unsigned __int128 carry = 0;
    for (int i = 0; i < n; ++i) {
        unsigned __int128 t = (unsigned __int128)x->d[i] + (i < y->len ? y->d[i] : 0) + carry;
        x->d[i] = (uint64_t)t;
        carry = t >> 64;
    }
    x->d[n] = (uint64_t)carry;
    x->len = n + 1;
    big_trim(x);
}
static int big_cmp(const big* x, const big* y) {
    if (x->len != y->len) return x->len < y->len ? -1 : 1;
    for (int i = x->len - 1; i >= 0; --i)
        if (x->d[i] != y->d[i]) return x->d[i] < y->d[i] ? -1 : 1;
    return 0;
}
/* x -= y, requires x >= y */
static void big_sub(big* x, const big* y) {
    uint64_t borrow = 0;
    for (int i = 0; i < x->len; ++i) {
        uint64_t yi = i < y->len ? y->d[i] : 0;
        uint64_t t = x->d[i] - yi;
        uint64_t b1 = x->d[i] < yi;
        uint64_t t2 = t - borrow;
        uint64_t b2 = t < borrow;
        x->d[i] = t2;
        borrow = b1 | b2;
    }
    big_trim(x);
}
/* x /= v; returns the remainder (0 when the division is exact) */
static uint64_t big_div_u64(big* x, uint64_t v) {
    unsigned __int128 rem = 0;
    for (int i = x->len - 1; i >= 0; --i) {
        unsigned __int128 cur = (rem << 64) | x->d[i];
        x->d[i] = (uint64_t)(cur / v);
        rem = cur % v;
    }
    big_trim(x);
    return (uint64_t)rem;
}
static int big_bits(const big* x) {
    if (x->len == 0) return 0;
    return 64 * (x->len - 1) + (64 - __builtin_clzll(x->d[x->len - 1]));
}
/* x ~= mant * 2^e with mant in [0.5, 1); the top 64 bits are kept (truncated),
 * so the relative error is below 2^-63.  Returns 0 for x == 0. */
static long double big_to_ld(const big* x, long* e) {
    int nb = big_bits(x);
    *e = 0;
    if (nb == 0) return 0.0L;
    uint64_t top;
    int sh = nb - 64; /* bit index of the lowest kept bit */
    if (sh <= 0) {
        top = x->d[0] << (-sh);
    } else {
        int w = sh / 64, b = sh % 64;
        top = x->d[w] >> b;
        if (b && w + 1 < x->len) top |= x->d[w + 1] << (64 - b);
    }
    *e = nb;
    return ldexpl((long double)top, -64);
}
/* x = u * v * 2^s */
static void big_from_spec(big* x, uint64_t u, uint64_t v, int s) {
    big_set_u64(x, u);
    big_mul_u64(x, v);
    big_shl(x, s);
}

/* ------------------------------------------------------------------------ */
/* Eq. (2), Sec. 2: R_nm(rho) = sum_s (-1)^s (n-s)! /                       */
/*        (s! ((n+m)/2-s)! ((n-m)/2-s)!) rho^(n-2s),   m >= 0, n-m even.    */
/* With k = (n-m)/2 and rho^2 = a/b (a, b positive integers):               */
/*   R = rho^m * b^-k * sum_s (-1)^s |c_s| b^s a^(k-s).                      */
/* The sum N' is an exact integer; it is evaluated by Horner in a, with the  */
/* positive and negative terms kept in two non-negative accumulators.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n, m, k;
    big* d;        /* d[s] = |c_s| * b^s, s = 0..k */
    long double bk_mant; long bk_exp;   /* b^k */
} zrp_col;

static int zrp_col_setup(zrp_col* c, int n, int m, const big* b) {
    c->n = n; c->m = m; c->k = (n - m) / 2;
    int k = c->k;
    int bb = big_bits(b);
    int cap = (int)((1.3 * n + 8 + (double)k * (bb + 1)) / 64.0) + 4;
    c->d = (big*)calloc((size_t)k + 1, sizeof(big));
    /* |c_0| = n! / ((k+m)! k!) = binomial(n, k), built by exact steps */
    big cur; big_init(&cur, cap);
    big_set_u64(&cur, 1);
    for (int i = 1; i <= k; ++i) {
        big_mul_u64(&cur, (uint64_t)(n - k + i));
        if (big_div_u64(&cur, (uint64_t)i) != 0) return -1;
    }
    /* d_0 = |c_0|; d_{s+1} = d_s * b * (k-s)(k+m-s) / ((s+1)(n-s)), exactly */
    big tmp; big_init(&tmp, cap);
    for (int s = 0; s <= k; ++s) {
        big_init(&c->d[s], cap);
        big_copy(&c->d[s], &cur);
        if (s == k) break;
        big_mul_u64(&cur, (uint64_t)(k - s) * (uint64_t)(k + m - s));
        big_mul(&tmp, &cur, b);
        big_copy(&cur, &tmp);
        if (big_div_u64(&cur, (uint64_t)(s + 1) * (uint64_t)(n - s)) != 0) return -1;
    }
    /* b^k */
    big_set_u64(&cur, 1);
    for (int s = 0; s < k; ++s) { big_mul(&tmp, &cur, b); big_copy(&cur, &tmp); }
    c->bk_mant = big_to_ld(&cur, &c->bk_exp);
    big_free(&cur); big_free(&tmp);
    return 0;
}
static void zrp_col_free(zrp_col* c) {
    for (int s = 0; s <= c->k; ++s) big_free(&c->d[s]);
    free(c->d);
}
/* R_nm at rho^2 = a/b; rho_ld = sqrt(a/b) in long double */
static double zrp_col_eval(const zrp_col* c, const big* a, long double rho_ld) {
    int k = c->k;
    int cap = c->d[0].len + 2;
    for (int s = 0; s <= k; ++s) if (c->d[s].len + 2 > cap) cap = c->d[s].len + 2;
    cap += (k + 1) * (a->len + 1) + 2;
    big E, O, t;
    big_init(&E, cap); big_init(&O, cap); big_init(&t, cap);
    for (int s = 0; s <= k; ++s) {
        if (s > 0) {
            big_mul(&t, &E, a); big_copy(&E, &t);
            big_mul(&t, &O, a); big_copy(&O, &t);
        }
        if ((s & 1) == 0) big_add(&E, &c->d[s]);
        else big_add(&O, &c->d[s]);
    }
    int sign = 1;
    if (big_cmp(&E, &O) >= 0) { big_sub(&E, &O); }
    else { big_sub(&O, &E); big_copy(&E, &O); sign = -1; }
    long e;
    long double mn = big_to_ld(&E, &e);
    big_free(&E); big_free(&O); big_free(&t);
    if (mn == 0.0L) return 0.0;
    long double q = ldexpl(mn / c->bk_mant, (int)(e - c->bk_exp));
    long double rm = (c->m == 0) ? 1.0L : powl(rho_ld, (long double)c->m);
    return (double)(sign * q * rm);
}

/* Evaluate R_nm (eq. (2)) at `count` points.  Point i has
 *   rho_i^2 = (ax[i] * ay[i] * 2^ash[i]) / (bx * by * 2^bsh).
 * out[i] receives R_nm(rho_i) rounded to FP64.  Returns 0, or -1 for bad
 * (n, m).  Requires a_i <= b (rho <= 1) for the documented accuracy. */
int zmo_zrp_column(int n, int m, uint64_t bx, uint64_t by, int bsh, int count,
                   const uint64_t* ax, const uint64_t* ay, const int* ash, double* out) {
    if (n < 0 || m < 0 || m > n || ((n - m) & 1)) return -1;
    big b; big_init(&b, 8);
    big_from_spec(&b, bx, by, bsh);
    long eb; long double mb = big_to_ld(&b, &eb);
    zrp_col c;
    if (zrp_col_setup(&c, n, m, &b) != 0) { big_free(&b); return -1; }
    big a; big_init(&a, 8);
    for (int i = 0; i < count; ++i) {
        big_from_spec(&a, ax[i], ay[i], ash[i]);
        long ea; long double ma = big_to_ld(&a, &ea);
        long double rho = (ma == 0.0L) ? 0.0L : sqrtl(ldexpl(ma / mb, (int)(ea - eb)));
        out[i] = zrp_col_eval(&c, &a, rho);
    }
    big_free(&a);
    zrp_col_free(&c);
    big_free(&b);
    return 0;
}

/* Canonical moment order: n = 0..nmax, then m = (n mod 2), (n mod 2)+2, ..., n. */
int zmo_num_moments(int nmax) {
    if (nmax < 0) return -1;
    int c = 0;
    for (int n = 0; n <= nmax; ++n)
        for (int m = n % 2; m <= n; m += 2) ++c;
    return c;
}
static void zmo_enumerate(int nmax, int* ns, int* ms) {
    int c = 0;
    for (int n = 0; n <= nmax; ++n)
        for (int m = n % 2; m <= n; m += 2) { ns[c] = n; ms[c] = m; ++c; }
}

/* R_nm for a list of (n, m) pairs at `count` points; out is [npairs][count].
 * Columns are independent and run in parallel. */
int zmo_zrp_pairs(int npairs, const int* ns, const int* ms, uint64_t bx, uint64_t by, int bsh,
                  int count, const uint64_t* ax, const uint64_t* ay, const int* ash, double* out) {
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int i = 0; i < npairs; ++i) {
        if (zmo_zrp_column(ns[i], ms[i], bx, by, bsh, count, ax, ay, ash, out + (size_t)i * count) != 0)
            bad = 1;
    }
    return bad ? -1 : 0;
}

/* The full table in canonical order, out is [M_tot][count]. */
int zmo_zrp_table(int nmax, uint64_t bx, uint64_t by, int bsh, int count, const uint64_t* ax,
                  const uint64_t* ay, const int* ash, double* out) {
    int mt = zmo_num_moments(nmax);
    if (mt < 0) return -1;
    int* ns = (int*)malloc(sizeof(int) * (size_t)mt);
    int* ms = (int*)malloc(sizeof(int) * (size_t)mt);
    zmo_enumerate(nmax, ns, ms);
    int rc = zmo_zrp_pairs(mt, ns, ms, bx, by, bsh, count, ax, ay, ash, out);
    free(ns); free(ms);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Polar image (Sec. 2.5): frame f is H x W, row-major.  The unit disk is   */
/* the frame's inscribed disk: radius D/2 pixels (D = min(H, W)), centre   */
/* ((W-1)/2, (H-1)/2) in pixel-centre coordinates, x to the right, y up,   */
/* theta counter-clockwise.  Sample (r, a) sits at rho = rho[r],           */
/* theta_a = 2 pi a / A; its value is the bilinear interpolation of the    */
/* four surrounding pixels, a pixel outside the frame counting as 0.        */
/* ------------------------------------------------------------------------ */
static double pix(const double* f, int H, int W, long i, long j) {
    if (i < 0 || j < 0 || i >= H || j >= W) return 0.0;
    return f[(size_t)i * W + j];
}
void zmo_resample(const double* f, int H, int W, int R, int A, const double* rho, double* fhat) {
    int D = H < W ? H : W;
    double rpx = 0.5 * D, cx = 0.5 * (W - 1), cy = 0.5 * (H - 1);
#pragma omp parallel for schedule(static)
    for (int r = 0; r < R; ++r) {
        double s = rho[r] * rpx;
        for (int a = 0; a < A; ++a) {
            double th = 2.0 * M_PI * (double)a / (double)A;
            double x = cx + s * cos(th);
            double y = cy - s * sin(th);
            double x0 = floor(x), y0 = floor(y);
            double fx = x - x0, fy = y - y0;
            long j = (long)x0, i = (long)y0;
            double v00 = pix(f, H, W, i, j), v01 = pix(f, H, W, i, j + 1);
            double v10 = pix(f, H, W, i + 1, j), v11 = pix(f, H, W, i + 1, j + 1);
            fhat[(size_t)r * A + a] =
                (1.0 - fy) * ((1.0 - fx) * v00 + fx * v01) + fy * ((1.0 - fx) * v10 + fx * v11);
        }
    }
}

/* Inner (angular) sum of eq. (1) on the uniform angle grid, a plain DFT:
 *   G[r][j] = sum_a fhat[r][a] * exp(-j m theta_a),  m = mlist[j],
 * stored as [R][nm][2] (re, im).  The phase table is indexed by the exact
 * integer (m * a) mod A. */
void zmo_angular_dft(const double* fhat, int R, int A, int nm, const int* mlist, double* G) {
    double* cs = (double*)malloc(sizeof(double) * 2 * (size_t)A);
    for (int j = 0; j < A; ++j) {
        double th = 2.0 * M_PI * (double)j / (double)A;
        cs[2 * j] = cos(th);
        cs[2 * j + 1] = sin(th);
    }
#pragma omp parallel for schedule(static)
    for (int r = 0; r < R; ++r) {
        const double* row = fhat + (size_t)r * A;
        for (int q = 0; q < nm; ++q) {
            long m = mlist[q];
            double re = 0.0, im = 0.0;
            for (int a = 0; a < A; ++a) {
                long j = (m * a) % A;
                re += row[a] * cs[2 * j];
                im -= row[a] * cs[2 * j + 1];
            }
            G[((size_t)r * nm + q) * 2] = re;
            G[((size_t)r * nm + q) * 2 + 1] = im;
        }
    }
    free(cs);
}

/* Outer (radial) sum of eq. (1) with the angle step 2 pi / A:
 *   Z_nm = (n+1)/(pi eps_m) * (2 pi / A) * sum_r w[r] R_nm(rho_r) G[r][m]
 * where w[r] is the radial quadrature weight (rho_r * drho for midpoint
 * rings) and eps_m is the Neumann factor of eq. (15) (2 for m = 0, else 1)
 * when `neumann` is set, 1 otherwise (eq. (14) vs eq. (1)).
 * Pair i is (ns[i], ms[i]); its angular sums are column cols[i] of G
 * ([R][nm][2]); table is [npairs][R]; Z is [npairs][2]. */
void zmo_radial_sum(const double* G, int R, int nm, int A, int npairs, const int* ns, const int* ms,
                    const int* cols, const double* table, const double* w, int neumann, double* Z) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < npairs; ++i) {
        int n = ns[i], m = ms[i], c = cols[i];
        double eps = (neumann && m == 0) ? 2.0 : 1.0;
        double re = 0.0, im = 0.0;
        for (int r = 0; r < R; ++r) {
            double t = w[r] * table[(size_t)i * R + r];
            re += t * G[((size_t)r * nm + c) * 2];
            im += t * G[((size_t)r * nm + c) * 2 + 1];
        }
        double k = (double)(n + 1) / (M_PI * eps) * (2.0 * M_PI / (double)A);
        Z[2 * i] = k * re;
        Z[2 * i + 1] = k * im;
    }
}

/* Eq. (3) with the first-order kernel of eq. (5): the Cartesian pixel sum
 *   Z~_nm = (n+1)/(pi eps_m) * Delta^2 * sum_{rho_xy <= 1} f(x,y) R_nm(rho_xy) exp(-j m theta_xy)
 * with Delta = 2/D (pixel width on the unit disk), pixel (i, j) at
 *   x = (2j - (W-1))/D, y = ((H-1) - 2i)/D,
 * so rho^2 = P/D^2 with the integer P = (2j-(W-1))^2 + ((H-1)-2i)^2.
 * Only moments with n <= nmax are computed; Z is [M_tot][2]. */
int zmo_cartesian(const double* f, int H, int W, int nmax, int neumann, double* Z) {
    int D = H < W ? H : W;
    long npx = 0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            long X = 2L * j - (W - 1), Y = (H - 1) - 2L * i;
            if (X * X + Y * Y <= (long)D * D) ++npx;
        }
    uint64_t* P = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(npx + 1));
    uint64_t* ones = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(npx + 1));
    int* zeros = (int*)calloc((size_t)(npx + 1), sizeof(int));
    double* val = (double*)malloc(sizeof(double) * (size_t)(npx + 1));
    double* th = (double*)malloc(sizeof(double) * (size_t)(npx + 1));
    long c = 0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            long X = 2L * j - (W - 1), Y = (H - 1) - 2L * i;
            if (X * X + Y * Y <= (long)D * D) {
                P[c] = (uint64_t)(X * X + Y * Y);
                ones[c] = 1;
                val[c] = f[(size_t)i * W + j];
                th[c] = atan2((double)Y, (double)X);
                ++c;
            }
        }
    int mt = zmo_num_moments(nmax);
    int* ns = (int*)malloc(sizeof(int) * (size_t)mt);
    int* ms = (int*)malloc(sizeof(int) * (size_t)mt);
    zmo_enumerate(nmax, ns, ms);
    double delta2 = (2.0 / D) * (2.0 / D);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int q = 0; q < mt; ++q) {
        double* rv = (double*)malloc(sizeof(double) * (size_t)(npx + 1));
        if (zmo_zrp_column(ns[q], ms[q], (uint64_t)D, (uint64_t)D, 0, (int)npx, P, ones, zeros, rv) != 0)
            bad = 1;
        double re = 0.0, im = 0.0;
        int m = ms[q];
        for (long p = 0; p < npx; ++p) {
            re += val[p] * rv[p] * cos(m * th[p]);
            im -= val[p] * rv[p] * sin(m * th[p]);
        }
        double eps = (neumann && m == 0) ? 2.0 : 1.0;
        double k = (double)(ns[q] + 1) / (M_PI * eps) * delta2;
        Z[2 * q] = k * re;
        Z[2 * q + 1] = k * im;
        free(rv);
    }
    free(P); free(ones); free(zeros); free(val); free(th); free(ns); free(ms);
    return bad ? -1 : 0;
}

/* One moment of the same Cartesian sum, Z~_nm for a single (n, m) with
 * |m| <= n and n - |m| even (m < 0 through Z_{n,-m} = conj(Z_nm), Sec. 2);
 * eq. (14) divides by the Neumann factor eps_m when `neumann` is set.  Z
 * receives (re, im).  Returns 0, or -1 for a bad (n, m). */
int zmo_cartesian_one(const double* f, int H, int W, int n, int m, int neumann, double* Z) {
    int am = m < 0 ? -m : m;
    if (n < 0 || am > n || ((n - am) & 1)) return -1;
    int D = H < W ? H : W;
    long npx = 0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            long X = 2L * j - (W - 1), Y = (H - 1) - 2L * i;
            if (X * X + Y * Y <= (long)D * D) ++npx;
        }
    uint64_t* P = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(npx + 1));
    uint64_t* ones = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(npx + 1));
    int* zeros = (int*)calloc((size_t)(npx + 1), sizeof(int));
    double* rv = (double*)malloc(sizeof(double) * (size_t)(npx + 1));
    long c = 0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            long X = 2L * j - (W - 1), Y = (H - 1) - 2L * i;
            if (X * X + Y * Y <= (long)D * D) {
                P[c] = (uint64_t)(X * X + Y * Y);
                ones[c] = 1;
                ++c;
            }
        }
    int rc = zmo_zrp_column(n, am, (uint64_t)D, (uint64_t)D, 0, (int)npx, P, ones, zeros, rv);
    double re = 0.0, im = 0.0;
    c = 0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            long X = 2L * j - (W - 1), Y = (H - 1) - 2L * i;
            if (X * X + Y * Y <= (long)D * D) {
                double th = atan2((double)Y, (double)X);
                double v = f[(size_t)i * W + j] * rv[c++];
                re += v * cos(am * th);
                im -= v * sin(am * th);
            }
        }
    double eps = (neumann && am == 0) ? 2.0 : 1.0;
    double k = (double)(n + 1) / (M_PI * eps) * (2.0 / D) * (2.0 / D);
    Z[0] = k * re;
    Z[1] = (m < 0 ? -k : k) * im;
    free(P); free(ones); free(zeros); free(rv);
    return rc;
}

/* Eq. (9): f~ = Re sum_n sum_{m=-n..n, n-m even} Z_nm R_nm(rho) exp(j m theta).
 * Only m >= 0 moments are stored; the m < 0 terms follow from
 * Z_{n,-m} = conj(Z_nm) (Sec. 2), so each m > 0 pair contributes
 * 2 Re(Z_nm exp(j m theta)) R_nm.  If the moments were divided by the
 * Neumann factor (eq. (14)), `neumann` multiplies eps_m back first.
 * If `one_sided` is set, the sum runs over m >= 0 only (each stored moment
 * once, no eps correction) -- the reconstruction the paper's Neumann
 * correction compensates for.
 * R is [M_tot][count] (R_nm at each point), theta is [count]. */
void zmo_reconstruct(const double* Z, int nmax, int neumann, int one_sided, int count,
                     const double* R, const double* theta, double* out) {
    int mt = zmo_num_moments(nmax);
    int* ns = (int*)malloc(sizeof(int) * (size_t)mt);
    int* ms = (int*)malloc(sizeof(int) * (size_t)mt);
    zmo_enumerate(nmax, ns, ms);
#pragma omp parallel for schedule(static)
    for (int p = 0; p < count; ++p) {
        double acc = 0.0;
        for (int i = 0; i < mt; ++i) {
            int m = ms[i];
            double zr = Z[2 * i], zi = Z[2 * i + 1];
            double term = zr * cos(m * theta[p]) - zi * sin(m * theta[p]);
            double rv = R[(size_t)i * count + p];
            if (one_sided) {
                acc += term * rv;
            } else {
                double eps = (neumann && m == 0) ? 2.0 : 1.0;
                acc += (m == 0 ? eps : 2.0) * term * rv;
            }
        }
        out[p] = acc;
    }
    free(ns); free(ms);
}

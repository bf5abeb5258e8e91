// dft_codelets.h -- small complex DFTs held entirely in registers.
//
//   X[k] = sum_{n<R} x[n] exp(S 2 pi i n k / R),  S = -1 or +1,  R <= 32.
//
// Primes 2, 3, 5 and the radix 4 are written out from the definition; sizes
// with coprime factors (6, 10, 12, 15, 18, 20, 24, 30) use the prime-factor
// mapping (no twiddles); 8, 9, 16, 25, 27 and 32 are split R = P*Q (P = 4
// when 4 | R and R > 4, else the smallest prime) by decimation in time with
// twiddles that are compile-time constants.
// The constants come from a constexpr sine/cosine: exact integer reduction of
// the angle numerator to the first half-quadrant, then a Taylor series.
#pragma once
#include <hip/hip_runtime.h>

namespace vloc {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x)
{
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 14; ++i) {
        term *= -x2 / double((2 * i) * (2 * i + 1));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x)
{
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 14; ++i) {
        term *= -x2 / double((2 * i - 1) * (2 * i));
        sum += term;
    }
    return sum;
}

struct CS {
    double c, s;
};

// cos and sin of 2 pi m / n.
constexpr CS cs_2pi(long m, long n)
{
    m %= n;
    if (m < 0) m += n;
    long q = (4 * m) / n;     // quadrant
    long r = 4 * m - q * n;   // angle = (pi/2) (q + r/n)
    double c = 1.0, s = 0.0;
    if (2 * r <= n) {
        double b = (kPi / 2) * double(r) / double(n);
        c = taylor_cos(b);
        s = taylor_sin(b);
    } else {
        double b = (kPi / 2) * double(n - r) / double(n);
        c = taylor_sin(b);
        s = taylor_cos(b);
    }
    switch (q) {
    case 0: return CS{c, s};
    case 1: return CS{-s, c};
    case 2: return CS{-c, -s};
    default: return CS{s, -c};
    }
}

// x *= exp(S 2 pi i m / n), with the trivial angles done without multiplies.
template <long M, long N, int S, typename T>
__host__ __device__ __forceinline__ void rot(T &xr, T &xi)
{
    constexpr long m = ((M % N) + N) % N;
    if constexpr (m == 0) {
        return;
    } else if constexpr (2 * m == N) {
        xr = -xr;
        xi = -xi;
    } else if constexpr (4 * m == N || 4 * m == 3 * N) {
        // exp(+- i pi/2): sign of the rotation is S for m = N/4, -S for 3N/4
        constexpr int sg = (4 * m == N) ? S : -S;
        T t = xr;
        if constexpr (sg > 0) { xr = -xi; xi = t; } else { xr = xi; xi = -t; }
    } else if constexpr (8 * m == N || 8 * m == 3 * N || 8 * m == 5 * N || 8 * m == 7 * N) {
        constexpr CS w = cs_2pi(m, N);
        constexpr T h = T(0.70710678118654752440084436210484904);
        constexpr T cr = w.c > 0 ? h : -h;
        constexpr T ci = (S > 0 ? w.s : -w.s) > 0 ? h : -h;
        // (xr + i xi)(cr + i ci) with |cr| = |ci| = h
        T a = xr, b = xi;
        if constexpr ((cr > 0) == (ci > 0)) {
            xr = cr * (a - b);
            xi = cr * (a + b);
        } else {
            xr = cr * (a + b);
            xi = cr * (b - a);
        }
    } else {
        constexpr CS w = cs_2pi(m, N);
        constexpr T wc = T(w.c);
        constexpr T ws = T(S > 0 ? w.s : -w.s);
        T a = xr, b = xi;
        xr = a * wc - b * ws;
        xi = a * ws + b * wc;
    }
}

template <int R, int S, typename T>
struct Dft;

template <int S, typename T>
struct Dft<1, S, T> {
    static __host__ __device__ __forceinline__ void run(T *, T *) {}
};

template <int S, typename T>
struct Dft<2, S, T> {
    static __host__ __device__ __forceinline__ void run(T *xr, T *xi)
    {
        T ar = xr[0] + xr[1], ai = xi[0] + xi[1];
        T br = xr[0] - xr[1], bi = xi[0] - xi[1];
        xr[0] = ar; xi[0] = ai; xr[1] = br; xi[1] = bi;
    }
};

template <int S, typename T>
struct Dft<3, S, T> {
    static __host__ __device__ __forceinline__ void run(T *xr, T *xi)
    {
        constexpr T s3 = T(S * 0.86602540378443864676372317075293618);
        T tr = xr[1] + xr[2], ti = xi[1] + xi[2];
        T ur = xr[0] - T(0.5) * tr, ui = xi[0] - T(0.5) * ti;
        T vr = s3 * (xr[1] - xr[2]), vi = s3 * (xi[1] - xi[2]);
        xr[0] = xr[0] + tr; xi[0] = xi[0] + ti;
        // X1 = u + i v, X2 = u - i v
        xr[1] = ur - vi; xi[1] = ui + vr;
        xr[2] = ur + vi; xi[2] = ui - vr;
    }
};

template <int S, typename T>
struct Dft<4, S, T> {
    static __host__ __device__ __forceinline__ void run(T *xr, T *xi)
    {
        T ar = xr[0] + xr[2], ai = xi[0] + xi[2];
        T br = xr[0] - xr[2], bi = xi[0] - xi[2];
        T cr = xr[1] + xr[3], ci = xi[1] + xi[3];
        T dr = xr[1] - xr[3], di = xi[1] - xi[3];
        // X1 = b + S i d, X3 = b - S i d
        xr[0] = ar + cr; xi[0] = ai + ci;
        xr[2] = ar - cr; xi[2] = ai - ci;
        if constexpr (S < 0) {
            xr[1] = br + di; xi[1] = bi - dr;
            xr[3] = br - di; xi[3] = bi + dr;
        } else {
            xr[1] = br - di; xi[1] = bi + dr;
            xr[3] = br + di; xi[3] = bi - dr;
        }
    }
};

template <int S, typename T>
struct Dft<5, S, T> {
    static __host__ __device__ __forceinline__ void run(T *xr, T *xi)
    {
        constexpr T c1 = T(0.30901699437494742410229341718281906);
        constexpr T c2 = T(-0.80901699437494742410229341718281906);
        constexpr T s1 = T(S * 0.95105651629515357211643933337938214);
        constexpr T s2 = T(S * 0.58778525229247312916870595463907277);
        T a1r = xr[1] + xr[4], a1i = xi[1] + xi[4];
        T b1r = xr[1] - xr[4], b1i = xi[1] - xi[4];
        T a2r = xr[2] + xr[3], a2i = xi[2] + xi[3];
        T b2r = xr[2] - xr[3], b2i = xi[2] - xi[3];
        T x0r = xr[0], x0i = xi[0];
        T p1r = x0r + c1 * a1r + c2 * a2r, p1i = x0i + c1 * a1i + c2 * a2i;
        T p2r = x0r + c2 * a1r + c1 * a2r, p2i = x0i + c2 * a1i + c1 * a2i;
        T q1r = s1 * b1r + s2 * b2r, q1i = s1 * b1i + s2 * b2i; // X1 = p1 + i q1
        T q2r = s2 * b1r - s1 * b2r, q2i = s2 * b1i - s1 * b2i; // X2 = p2 + i q2
        xr[0] = x0r + a1r + a2r; xi[0] = x0i + a1i + a2i;
        xr[1] = p1r - q1i; xi[1] = p1i + q1r;
        xr[4] = p1r + q1i; xi[4] = p1i - q1r;
        xr[2] = p2r - q2i; xi[2] = p2i + q2r;
        xr[3] = p2r + q2i; xi[3] = p2i - q2r;
    }
};

constexpr int split_factor(int R)
{
    if (R % 4 == 0 && R > 4) return 4;
    if (R % 2 == 0) return 2;
    if (R % 3 == 0) return 3;
    if (R % 5 == 0) return 5;
    return R;
}

// Decimation in time: n = P n' + r, X[k + Q q] = sum_r W_R^{r k} W_P^{r q} Y_r[k],
// Y_r = DFT_Q(x[P n' + r]).
template <int R, int S, typename T>
struct Dft {
    static constexpr int P = split_factor(R);
    static constexpr int Q = R / P;
    static_assert(P > 1 && Q > 1, "codelet size must be composite here");

    template <int r>
    static __host__ __device__ __forceinline__ void sub(const T *xr, const T *xi, T (*yr)[Q], T (*yi)[Q])
    {
#pragma unroll
        for (int n = 0; n < Q; ++n) {
            yr[r][n] = xr[P * n + r];
            yi[r][n] = xi[P * n + r];
        }
        Dft<Q, S, T>::run(yr[r], yi[r]);
    }

    template <int r, int k>
    static __host__ __device__ __forceinline__ void tw(T (*yr)[Q], T (*yi)[Q])
    {
        rot<r * k, R, S, T>(yr[r][k], yi[r][k]);
    }

    template <int r>
    static __host__ __device__ __forceinline__ void tw_row(T (*yr)[Q], T (*yi)[Q])
    {
        tw_k<r, 0>(yr, yi);
    }
    template <int r, int k>
    static __host__ __device__ __forceinline__ void tw_k(T (*yr)[Q], T (*yi)[Q])
    {
        if constexpr (k < Q) {
            tw<r, k>(yr, yi);
            tw_k<r, k + 1>(yr, yi);
        }
    }
    template <int r>
    static __host__ __device__ __forceinline__ void all_sub(const T *xr, const T *xi, T (*yr)[Q], T (*yi)[Q])
    {
        if constexpr (r < P) {
            sub<r>(xr, xi, yr, yi);
            tw_row<r>(yr, yi);
            all_sub<r + 1>(xr, xi, yr, yi);
        }
    }

    static __host__ __device__ __forceinline__ void run(T *xr, T *xi)
    {
        T yr[P][Q], yi[P][Q];
        all_sub<0>(xr, xi, yr, yi);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            T zr[P], zi[P];
#pragma unroll
            for (int r = 0; r < P; ++r) {
                zr[r] = yr[r][k];
                zi[r] = yi[r][k];
            }
            Dft<P, S, T>::run(zr, zi);
#pragma unroll
            for (int q = 0; q < P; ++q) {
                xr[k + Q * q] = zr[q];
                xi[k + Q * q] = zi[q];
            }
        }
    }
};

// Prime-factor (Good-Thomas) split of R = A B with gcd(A, B) = 1: with the
// input index n = (B n1 + A n2) mod R and the output index
// k = (B (B^-1 mod A) k1 + A (A^-1 mod B) k2) mod R the DFT becomes an A x B
// two-dimensional DFT with no twiddle factors.
constexpr int inv_mod(int a, int m)
{
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}

template <int A, int B, int S, typename T>
struct Pfa {
    static __host__ __device__ __forceinline__ void run(T *xr, T *xi)
    {
        constexpr int R = A * B;
        constexpr int ka = B * inv_mod(B, A), kb = A * inv_mod(A, B);
        T yr[A][B], yi[A][B];
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) {
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) {
                yr[n1][n2] = xr[(B * n1 + A * n2) % R];
                yi[n1][n2] = xi[(B * n1 + A * n2) % R];
            }
            Dft<B, S, T>::run(yr[n1], yi[n1]);
        }
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            T zr[A], zi[A];
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) {
                zr[n1] = yr[n1][k2];
                zi[n1] = yi[n1][k2];
            }
            Dft<A, S, T>::run(zr, zi);
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) {
                xr[(ka * k1 + kb * k2) % R] = zr[k1];
                xi[(ka * k1 + kb * k2) % R] = zi[k1];
            }
        }
    }
};

// Sizes with coprime factors use the prime-factor split.
template <int S, typename T>
struct Dft<6, S, T> : Pfa<2, 3, S, T> {};
template <int S, typename T>
struct Dft<10, S, T> : Pfa<2, 5, S, T> {};
template <int S, typename T>
struct Dft<12, S, T> : Pfa<4, 3, S, T> {};
template <int S, typename T>
struct Dft<15, S, T> : Pfa<3, 5, S, T> {};
template <int S, typename T>
struct Dft<18, S, T> : Pfa<2, 9, S, T> {};
template <int S, typename T>
struct Dft<20, S, T> : Pfa<4, 5, S, T> {};
template <int S, typename T>
struct Dft<24, S, T> : Pfa<8, 3, S, T> {};
template <int S, typename T>
struct Dft<30, S, T> : Pfa<2, 15, S, T> {};

// Sizes a plan may use for the two factors of a line length.
__host__ __device__ constexpr bool codelet_supported(int R)
{
    return R == 1 || R == 2 || R == 3 || R == 4 || R == 5 || R == 6 || R == 8 || R == 9 ||
           R == 10 || R == 12 || R == 15 || R == 16 || R == 18 || R == 20 || R == 24 ||
           R == 25 || R == 27 || R == 30 || R == 32;
}

} // namespace vloc

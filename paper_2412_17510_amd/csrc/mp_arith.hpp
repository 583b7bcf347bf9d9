// mp_arith.hpp -- device multi-component arithmetic for gfx950 (header-only HIP).
//
// Error-free transformations and the double-double / triple-double / quad-double
// operations of Kouya, arXiv 2412.17510, Sec. 2, on binary64 VALU instructions:
//   * TwoSum (6 flops), QuickTwoSum (3), TwoProd via one v_fma_f64 (2);
//   * DD add and multiply exactly as Algorithms 1 and 2; DD times binary64 as
//     Algorithm 3 with the trailing product restored;
//   * QD "sloppy" add and multiply after Hida, Li and Bailey (the paper's QD basis):
//     componentwise/levelled partial results merged by ThreeSum / ThreeSum2 and a
//     5-to-4 renormalisation;
//   * TD = the QD operations with the fourth component of both operands zero,
//     keeping three components (Sec. 2, TD paragraph).
//
// The library is compiled with -ffp-contract=off: every + and * below is a single
// rounded binary64 operation, and the only fused operation is the explicit FMA in
// TwoProd (where it yields the exact product error).  The operation sequences are
// the normative ones of the library; a change here changes results bitwise.
#pragma once

#include <hip/hip_runtime.h>

namespace mpk {

template <int K>
struct mpn {
    double c[K];
};

using dd_t = mpn<2>;
using td_t = mpn<3>;
using qd_t = mpn<4>;

// ---------------------------------------------------------------------------
// error-free transformations
// ---------------------------------------------------------------------------

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    const double sum = a + b;
    const double bv = sum - a;
    const double av = sum - bv;
    e = (a - av) + (b - bv);
    s = sum;
}

__device__ __forceinline__ void quick_two_sum(double a, double b, double &s, double &e)
{
    const double sum = a + b;
    e = b - (sum - a);
    s = sum;
}

__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e)
{
    const double prod = a * b;
    e = __builtin_fma(a, b, -prod);
    p = prod;
}

// ---------------------------------------------------------------------------
// double-double (Algorithms 1, 2, 3)
// ---------------------------------------------------------------------------

__device__ __forceinline__ dd_t dd_add(const dd_t &x, const dd_t &y)
{
    double s, e;
    two_sum(x.c[0], y.c[0], s, e);
    const double w = x.c[1] + y.c[1];
    e = e + w;
    dd_t r;
    quick_two_sum(s, e, r.c[0], r.c[1]);
    return r;
}

__device__ __forceinline__ dd_t dd_mul(const dd_t &x, const dd_t &y)
{
    double p1, p2;
    two_prod(x.c[0], y.c[0], p1, p2);
    const double w1 = x.c[0] * y.c[1];
    const double w2 = x.c[1] * y.c[0];
    const double w3 = w1 + w2;
    p2 = p2 + w3;
    dd_t r;
    quick_two_sum(p1, p2, r.c[0], r.c[1]);
    return r;
}

__device__ __forceinline__ dd_t dd_mul_d(const dd_t &x, double y)
{
    double p1, p2;
    two_prod(x.c[0], y, p1, p2);
    const double w = x.c[1] * y;
    p2 = w + p2;
    dd_t r;
    quick_two_sum(p1, p2, r.c[0], r.c[1]);
    return r;
}

// DD comparison a <= b (non-overlapping pairs: compare leading, then trailing parts)
__device__ __forceinline__ bool dd_le(const dd_t &a, const dd_t &b)
{
    return (a.c[0] < b.c[0]) || (a.c[0] == b.c[0] && a.c[1] <= b.c[1]);
}

// DD division a / b (Dekker's long division): q1 = a0 / b0; the remainder a - q1 b
// from an exact product q1*b0, the trailing products and an exact difference;
// q2 = remainder / b0; result QuickTwoSum(q1, q2).  Binary64 division is the
// correctly rounded IEEE operation.
__device__ __forceinline__ dd_t dd_div(const dd_t &a, const dd_t &b)
{
    const double q1 = a.c[0] / b.c[0];
    double p, e;
    two_prod(q1, b.c[0], p, e);
    const double w = q1 * b.c[1];
    e = e + w;
    double s, f;
    two_sum(a.c[0], -p, s, f);
    f = f - e;
    f = f + a.c[1];
    const double q2 = (s + f) / b.c[0];
    dd_t r;
    quick_two_sum(q1, q2, r.c[0], r.c[1]);
    return r;
}

// ---------------------------------------------------------------------------
// quad-double building blocks
// ---------------------------------------------------------------------------

// (a, b, c) -> (s, e1, e2), s + e1 + e2 == a + b + c exactly
__device__ __forceinline__ void three_sum(double a, double b, double c, double &s, double &e1, double &e2)
{
    double t1, t2, t3;
    two_sum(a, b, t1, t2);
    two_sum(c, t1, s, t3);
    two_sum(t2, t3, e1, e2);
}

// (a, b, c) -> (s, e1): the two error levels merged by one rounded add
__device__ __forceinline__ void three_sum2(double a, double b, double c, double &s, double &e1)
{
    double t1, t2, t3;
    two_sum(a, b, t1, t2);
    two_sum(c, t1, s, t3);
    e1 = t2 + t3;
}

// Renormalise five roughly ordered terms into four non-overlapping components.
// Bottom-up QuickTwoSum sweep to (t0; t1..t4), then a top-down sweep that closes a
// component whenever the running QuickTwoSum error is non-zero, at most three times;
// the final carry is the last component.  The all-non-zero case (the usual one for
// data with full-length mantissas) takes a straight path; any lane with a zero error
// takes the general select-based path, which gives the same values.
//
// KEEP = 3 (triple-double: only three components are read) widens the straight path.
// With t1 and the second closing error e2 non-zero, the general path closes t0 and s2
// and its third component is s3 when the third closing error e3 is non-zero, else the
// QuickTwoSum sum fl(s3 + t4) (e3 = 0 carries s3 on to t4).  The straight path selects
// between the two: the same three values, without the general path, which zero-padded
// fourth components would otherwise send many lanes down.
template <int KEEP = 4>
__device__ __forceinline__ qd_t renorm5(double c0, double c1, double c2, double c3, double c4)
{
    double s, t0, t1, t2, t3, t4;
    quick_two_sum(c3, c4, s, t4);
    quick_two_sum(c2, s, s, t3);
    quick_two_sum(c1, s, s, t2);
    quick_two_sum(c0, s, t0, t1);

    qd_t r;
    double s2, e2, s3, e3;
    quick_two_sum(t1, t2, s2, e2);
    quick_two_sum(e2, t3, s3, e3);
    if constexpr (KEEP == 3) {
        if (__builtin_expect((t1 != 0.0) & (e2 != 0.0), 1)) {
            r.c[0] = t0;
            r.c[1] = s2;
            r.c[2] = (e3 != 0.0) ? s3 : s3 + t4;
            r.c[3] = 0.0;
            return r;
        }
    } else {
        if (__builtin_expect((t1 != 0.0) & (e2 != 0.0) & (e3 != 0.0), 1)) {
            r.c[0] = t0;
            r.c[1] = s2;
            r.c[2] = s3;
            r.c[3] = e3 + t4;
            return r;
        }
    }
    // general path: carry s, k components closed so far
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
    int k = 0;
    s = t0;
    if (t1 != 0.0) {
        r0 = t0;
        k = 1;
        s = t1;
    }
    const double ts[3] = {t2, t3, t4};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double sn, e;
        quick_two_sum(s, ts[i], sn, e);
        s = sn;
        const bool close = (e != 0.0) & (k < 3);
        if (close) {
            r0 = (k == 0) ? s : r0;
            r1 = (k == 1) ? s : r1;
            r2 = (k == 2) ? s : r2;
            s = e;
            k = k + 1;
        }
    }
    r0 = (k == 0) ? s : r0;
    r1 = (k == 1) ? s : r1;
    r2 = (k == 2) ? s : r2;
    r3 = (k == 3) ? s : r3;
    r.c[0] = r0;
    r.c[1] = r1;
    r.c[2] = r2;
    r.c[3] = r3;
    return r;
}

// QD sloppy addition (KEEP = 3: only the first three components are meaningful)
template <int KEEP = 4>
__device__ __forceinline__ qd_t qd_add(const qd_t &x, const qd_t &y)
{
    double s0, s1, s2, s3, e0, e1, e2, e3;
    two_sum(x.c[0], y.c[0], s0, e0);
    two_sum(x.c[1], y.c[1], s1, e1);
    two_sum(x.c[2], y.c[2], s2, e2);
    two_sum(x.c[3], y.c[3], s3, e3);
    two_sum(s1, e0, s1, e0);                // order eps
    three_sum(s2, e0, e1, s2, e0, e1);      // order eps^2
    three_sum2(s3, e0, e2, s3, e0);         // order eps^3
    double t = e0 + e1;                     // order eps^4
    t = t + e3;
    return renorm5<KEEP>(s0, s1, s2, s3, t);
}

// QD sloppy multiplication (KEEP = 3: only the first three components are meaningful)
template <int KEEP = 4>
__device__ __forceinline__ qd_t qd_mul(const qd_t &x, const qd_t &y)
{
    double p0, q0, p1, q1, p2, q2, p3, q3, p4, q4, p5, q5;
    two_prod(x.c[0], y.c[0], p0, q0);       // order 1
    two_prod(x.c[0], y.c[1], p1, q1);       // order eps
    two_prod(x.c[1], y.c[0], p2, q2);
    two_prod(x.c[0], y.c[2], p3, q3);       // order eps^2
    two_prod(x.c[1], y.c[1], p4, q4);
    two_prod(x.c[2], y.c[0], p5, q5);
    double h1, m1, l1;
    three_sum(p1, p2, q0, h1, m1, l1);      // order eps
    double u0, u1, u2, v0, v1, v2;
    three_sum(m1, q1, q2, u0, u1, u2);      // order eps^2: two ThreeSums ...
    three_sum(p3, p4, p5, v0, v1, v2);
    double s0, f0, s1, f1;
    two_sum(u0, v0, s0, f0);                // ... merged level by level
    two_sum(u1, v1, s1, f1);
    double s2 = u2 + v2;
    two_sum(s1, f0, s1, f0);
    s2 = s2 + (f0 + f1);
    double t = x.c[0] * y.c[3];             // order eps^3
    t = t + x.c[1] * y.c[2];
    t = t + x.c[2] * y.c[1];
    t = t + x.c[3] * y.c[0];
    t = t + l1;
    t = t + q3;
    t = t + q4;
    t = t + q5;
    s1 = s1 + t;
    return renorm5<KEEP>(p0, h1, s0, s1, s2);
}

// QD times binary64 (Alg. 4; its garbled steps read after Hida, Li and Bailey's
// product of a quad-double by a double): the three leading partial products exact,
// the fourth plain; the order-eps pair merged by TwoSum, the order-eps^2 terms by
// ThreeSum, the first order-eps^2 error with the second product error and the
// fourth product by ThreeSum2, the last two errors by one add; renormalised.
template <int KEEP = 4>
__device__ __forceinline__ qd_t qd_mul_d(const qd_t &x, double y)
{
    double p0, q0, p1, q1, p2, q2;
    two_prod(x.c[0], y, p0, q0);
    two_prod(x.c[1], y, p1, q1);
    two_prod(x.c[2], y, p2, q2);
    const double p3 = x.c[3] * y;
    double s1, s2;
    two_sum(q0, p1, s1, s2);
    double t0, t1, t2;
    three_sum(s2, q1, p2, t0, t1, t2);
    double u0, u1;
    three_sum2(t1, q2, p3, u0, u1);
    return renorm5<KEEP>(p0, s1, t0, u0, u1 + t2);
}

// ---------------------------------------------------------------------------
// triple-double: QD with zero fourth components, three components kept
// ---------------------------------------------------------------------------

__device__ __forceinline__ td_t td_add(const td_t &x, const td_t &y)
{
    const qd_t a = {{x.c[0], x.c[1], x.c[2], 0.0}};
    const qd_t b = {{y.c[0], y.c[1], y.c[2], 0.0}};
    const qd_t r = qd_add<3>(a, b);
    return td_t{{r.c[0], r.c[1], r.c[2]}};
}

__device__ __forceinline__ td_t td_mul(const td_t &x, const td_t &y)
{
    const qd_t a = {{x.c[0], x.c[1], x.c[2], 0.0}};
    const qd_t b = {{y.c[0], y.c[1], y.c[2], 0.0}};
    const qd_t r = qd_mul<3>(a, b);
    return td_t{{r.c[0], r.c[1], r.c[2]}};
}

// TD times binary64 (Alg. 5): the QD product of the zero-padded value, three
// components kept
__device__ __forceinline__ td_t td_mul_d(const td_t &x, double y)
{
    const qd_t a = {{x.c[0], x.c[1], x.c[2], 0.0}};
    const qd_t r = qd_mul_d<3>(a, y);
    return td_t{{r.c[0], r.c[1], r.c[2]}};
}

// ---------------------------------------------------------------------------
// K-generic dispatch
// ---------------------------------------------------------------------------

__device__ __forceinline__ dd_t mp_mul_d(const dd_t &x, double y) { return dd_mul_d(x, y); }
__device__ __forceinline__ td_t mp_mul_d(const td_t &x, double y) { return td_mul_d(x, y); }
__device__ __forceinline__ qd_t mp_mul_d(const qd_t &x, double y) { return qd_mul_d(x, y); }

__device__ __forceinline__ dd_t mp_add(const dd_t &x, const dd_t &y) { return dd_add(x, y); }
__device__ __forceinline__ td_t mp_add(const td_t &x, const td_t &y) { return td_add(x, y); }
__device__ __forceinline__ qd_t mp_add(const qd_t &x, const qd_t &y) { return qd_add(x, y); }
__device__ __forceinline__ dd_t mp_mul(const dd_t &x, const dd_t &y) { return dd_mul(x, y); }
__device__ __forceinline__ td_t mp_mul(const td_t &x, const td_t &y) { return td_mul(x, y); }
__device__ __forceinline__ qd_t mp_mul(const qd_t &x, const qd_t &y) { return qd_mul(x, y); }

template <int K>
__device__ __forceinline__ mpn<K> mp_neg(const mpn<K> &x)
{
    mpn<K> r;
#pragma unroll
    for (int c = 0; c < K; ++c) r.c[c] = -x.c[c];
    return r;
}

template <int K>
__device__ __forceinline__ mpn<K> mp_zero()
{
    mpn<K> r;
#pragma unroll
    for (int c = 0; c < K; ++c) r.c[c] = 0.0;
    return r;
}

}  // namespace mpk

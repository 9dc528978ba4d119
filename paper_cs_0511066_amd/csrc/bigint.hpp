// Host big integers for the reconstruction steps (Chinese remaindering,
// p-adic to integer conversion, rational reconstruction, the final product
// det = s_n * (det / s_n)).  Sign + magnitude, base 2^64 limbs, schoolbook
// multiplication with a Karatsuba split for long operands, Knuth long
// division.  Exceptions never leave the library (the C-ABI layer catches).
#pragma once
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

namespace dethost {

typedef unsigned __int128 u128;

class BigInt {
 public:
  int sign = 0;                  // -1, 0, +1
  std::vector<uint64_t> mag;     // little-endian, no leading zero limb

  BigInt() {}
  static BigInt from_i64(int64_t v) {
    BigInt r;
    if (v == 0) return r;
    r.sign = v < 0 ? -1 : 1;
    r.mag.push_back(v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v);
    return r;
  }
  static BigInt from_u64(uint64_t v) {
    BigInt r;
    if (v) { r.sign = 1; r.mag.push_back(v); }
    return r;
  }
  bool is_zero() const { return sign == 0; }
  void trim() {
    while (!mag.empty() && mag.back() == 0) mag.pop_back();
    if (mag.empty()) sign = 0;
  }
  int64_t bit_length() const {
    if (mag.empty()) return 0;
    return (int64_t)(mag.size() - 1) * 64 + (64 - __builtin_clzll(mag.back()));
  }

  // ---- magnitude helpers
  static int cmp_mag(const std::vector<uint64_t>& a, const std::vector<uint64_t>& b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
      if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
  }
  static void add_mag(std::vector<uint64_t>& out, const std::vector<uint64_t>& a,
                      const std::vector<uint64_t>& b) {
    const std::vector<uint64_t>& x = a.size() >= b.size() ? a : b;
    const std::vector<uint64_t>& y = a.size() >= b.size() ? b : a;
    std::vector<uint64_t> r(x.size() + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < x.size(); i++) {
      u128 s = (u128)x[i] + (i < y.size() ? y[i] : 0) + c;
      r[i] = (uint64_t)s;
      c = (uint64_t)(s >> 64);
    }
    r[x.size()] = c;
    out.swap(r);
    while (!out.empty() && out.back() == 0) out.pop_back();
  }
  // a - b with |a| >= |b|
  static void sub_mag(std::vector<uint64_t>& out, const std::vector<uint64_t>& a,
                      const std::vector<uint64_t>& b) {
    std::vector<uint64_t> r(a.size());
    uint64_t br = 0;
    for (size_t i = 0; i < a.size(); i++) {
      uint64_t bi = i < b.size() ? b[i] : 0;
      u128 d = (u128)a[i] - bi - br;
      r[i] = (uint64_t)d;
      br = (uint64_t)(d >> 127);   // 1 if the subtraction wrapped
    }
    out.swap(r);
    while (!out.empty() && out.back() == 0) out.pop_back();
  }
  static void mul_school(uint64_t* out, const uint64_t* a, size_t na, const uint64_t* b, size_t nb) {
    std::fill(out, out + na + nb, 0);
    for (size_t i = 0; i < na; i++) {
      uint64_t c = 0;
      const uint64_t ai = a[i];
      if (!ai) continue;
      for (size_t j = 0; j < nb; j++) {
        u128 t = (u128)ai * b[j] + out[i + j] + c;
        out[i + j] = (uint64_t)t;
        c = (uint64_t)(t >> 64);
      }
      out[i + nb] = c;
    }
  }
  static std::vector<uint64_t> mul_mag(const std::vector<uint64_t>& a,
                                       const std::vector<uint64_t>& b) {
    if (a.empty() || b.empty()) return {};
    std::vector<uint64_t> r(a.size() + b.size());
    if (a.size() < 48 || b.size() < 48) {
      mul_school(r.data(), a.data(), a.size(), b.data(), b.size());
    } else {
      // Karatsuba on the longer operand split at h limbs
      const size_t h = std::max(a.size(), b.size()) / 2;
      auto lo = [h](const std::vector<uint64_t>& v) {
        std::vector<uint64_t> o(v.begin(), v.begin() + std::min(h, v.size()));
        while (!o.empty() && o.back() == 0) o.pop_back();
        return o;
      };
      auto hi = [h](const std::vector<uint64_t>& v) {
        std::vector<uint64_t> o;
        if (v.size() > h) o.assign(v.begin() + h, v.end());
        return o;
      };
      std::vector<uint64_t> a0 = lo(a), a1 = hi(a), b0 = lo(b), b1 = hi(b);
      std::vector<uint64_t> z0 = mul_mag(a0, b0), z2 = mul_mag(a1, b1), sa, sb;
      add_mag(sa, a0, a1);
      add_mag(sb, b0, b1);
      std::vector<uint64_t> z1 = mul_mag(sa, sb);
      sub_mag(z1, z1, z0);
      sub_mag(z1, z1, z2);
      std::fill(r.begin(), r.end(), 0);
      auto acc = [&r](const std::vector<uint64_t>& v, size_t shift) {
        uint64_t c = 0;
        size_t i = 0;
        for (; i < v.size(); i++) {
          u128 s = (u128)r[i + shift] + v[i] + c;
          r[i + shift] = (uint64_t)s;
          c = (uint64_t)(s >> 64);
        }
        for (size_t k = i + shift; c && k < r.size(); k++) {
          u128 s = (u128)r[k] + c;
          r[k] = (uint64_t)s;
          c = (uint64_t)(s >> 64);
        }
      };
      acc(z0, 0);
      acc(z1, h);
      acc(z2, 2 * h);
    }
    while (!r.empty() && r.back() == 0) r.pop_back();
    return r;
  }

  // ---- signed arithmetic
  friend BigInt operator+(const BigInt& a, const BigInt& b) {
    if (a.sign == 0) return b;
    if (b.sign == 0) return a;
    BigInt r;
    if (a.sign == b.sign) {
      add_mag(r.mag, a.mag, b.mag);
      r.sign = a.sign;
    } else {
      int c = cmp_mag(a.mag, b.mag);
      if (c == 0) return BigInt();
      if (c > 0) { sub_mag(r.mag, a.mag, b.mag); r.sign = a.sign; }
      else { sub_mag(r.mag, b.mag, a.mag); r.sign = b.sign; }
    }
    r.trim();
    return r;
  }
  BigInt operator-() const { BigInt r = *this; r.sign = -r.sign; return r; }
  friend BigInt operator-(const BigInt& a, const BigInt& b) { return a + (-b); }
  friend BigInt operator*(const BigInt& a, const BigInt& b) {
    BigInt r;
    if (a.sign == 0 || b.sign == 0) return r;
    r.mag = mul_mag(a.mag, b.mag);
    r.sign = a.sign * b.sign;
    r.trim();
    return r;
  }
  // this = this * m + c  (m, c small, this >= 0 or any sign with c of same meaning)
  void mul_add_small(uint64_t m, uint64_t c) {
    if (sign < 0) {   // general path for negative values
      *this = *this * from_u64(m) + from_u64(c);
      return;
    }
    uint64_t carry = c;
    for (size_t i = 0; i < mag.size(); i++) {
      u128 t = (u128)mag[i] * m + carry;
      mag[i] = (uint64_t)t;
      carry = (uint64_t)(t >> 64);
    }
    if (carry) mag.push_back(carry);
    sign = mag.empty() ? 0 : 1;
    trim();
  }
  // this = this * m + c for this >= 0, m < 2^63 and c < 2^127 (two base-p
  // digits a pass in a radix conversion); every partial sum is below 2^128.
  void mul_add_u128(uint64_t m, u128 c) {
    u128 carry = c;
    for (size_t i = 0; i < mag.size(); i++) {
      const u128 t = (u128)mag[i] * m + carry;
      mag[i] = (uint64_t)t;
      carry = t >> 64;
    }
    while (carry) {
      mag.push_back((uint64_t)carry);
      carry >>= 64;
    }
    sign = mag.empty() ? 0 : 1;
    trim();
  }
  // Sign-magnitude linear combination in place:
  //   (x, y) <- (A x + B y, C x + D y)
  // for 64-bit signed cofactors (|A|, |B|, |C|, |D| < 2^63), one pass over the
  // words per result with 128-bit accumulation: terms of equal sign add as
  // magnitudes (below 2^128 with the carry), terms of opposite sign subtract
  // (below 2^127 in magnitude); a negative result is negated at the end.
  // (x, y) <- (A x + B y, C x + D y) for |A|, |B|, |C|, |D| < 2^62, in place
  // and in one pass: limb i of both results needs only limb i of x and y
  // and the running carries (two's complement, 128-bit: |a x_i + b y_i| <
  // 2^127), so each is written over the inputs' limb i.
  static void lincomb2(BigInt& x, BigInt& y, int64_t A, int64_t B, int64_t C, int64_t D) {
    const int64_t a = x.sign < 0 ? -A : A, b = y.sign < 0 ? -B : B;
    const int64_t c = x.sign < 0 ? -C : C, d = y.sign < 0 ? -D : D;
    const size_t n = std::max(x.mag.size(), y.mag.size());
    x.mag.resize(n + 1, 0);
    y.mag.resize(n + 1, 0);
    // the signs of the four coefficients select one of 16 loops, so that
    // every product is one unsigned 64 x 64 -> 128 multiplication
    const int sel = (a < 0) << 3 | (b < 0) << 2 | (c < 0) << 1 | (d < 0);
    const uint64_t ma = mag64(a), mb = mag64(b), mc = mag64(c), md = mag64(d);
    __int128 c1 = 0, c2 = 0;
    switch (sel) {
#define LC_CASE(k) \
      case k: lc_loop<(k >> 3) & 1, (k >> 2) & 1, (k >> 1) & 1, k & 1>(x.mag.data(), y.mag.data(), n, ma, mb, mc, md, c1, c2); break;
      LC_CASE(0) LC_CASE(1) LC_CASE(2) LC_CASE(3) LC_CASE(4) LC_CASE(5) LC_CASE(6) LC_CASE(7)
      LC_CASE(8) LC_CASE(9) LC_CASE(10) LC_CASE(11) LC_CASE(12) LC_CASE(13) LC_CASE(14) LC_CASE(15)
#undef LC_CASE
    }
    // the carries are below 2^63 in magnitude: one more limb each, and the
    // sign of the result is the sign of that limb
    x.mag[n] = (uint64_t)c1;
    y.mag[n] = (uint64_t)c2;
    finish_twos(x, c1 < 0);
    finish_twos(y, c2 < 0);
  }
  static uint64_t mag64(int64_t v) { return v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v; }
  template <bool NA, bool NB, bool NC, bool ND>
  static void lc_loop(uint64_t* xm, uint64_t* ym, size_t n, uint64_t ma, uint64_t mb, uint64_t mc,
                      uint64_t md, __int128& c1, __int128& c2) {
    for (size_t i = 0; i < n; i++) {
      const uint64_t xi = xm[i], yi = ym[i];
      // |coefficient| < 2^62: each product is below 2^126, and so is their
      // signed sum plus the carry, which fits a signed 128-bit word
      const __int128 pa = (__int128)((u128)xi * ma), pb = (__int128)((u128)yi * mb);
      const __int128 pc = (__int128)((u128)xi * mc), pd = (__int128)((u128)yi * md);
      const __int128 t1 = (NA ? -pa : pa) + (NB ? -pb : pb) + c1;
      const __int128 t2 = (NC ? -pc : pc) + (ND ? -pd : pd) + c2;
      xm[i] = (uint64_t)t1;
      ym[i] = (uint64_t)t2;
      c1 = t1 >> 64;
      c2 = t2 >> 64;
    }
  }
  // x.mag holds a two's complement value (its top limb gives the sign):
  // back to sign and magnitude
  static void finish_twos(BigInt& x, bool neg) {
    if (neg) {
      uint64_t cy = 1;
      for (auto& w : x.mag) {
        const u128 t = (u128)(~w) + cy;
        w = (uint64_t)t;
        cy = (uint64_t)(t >> 64);
      }
    }
    x.sign = neg ? -1 : 1;
    x.trim();
  }
  static BigInt combine(const BigInt& x, int64_t a, const BigInt& y, int64_t b) {
    const int sa = x.sign * (a < 0 ? -1 : a > 0 ? 1 : 0);
    const int sb = y.sign * (b < 0 ? -1 : b > 0 ? 1 : 0);
    const uint64_t ma = a < 0 ? (uint64_t)0 - (uint64_t)a : (uint64_t)a;
    const uint64_t mb = b < 0 ? (uint64_t)0 - (uint64_t)b : (uint64_t)b;
    BigInt r;
    if (sa == 0 && sb == 0) return r;
    const size_t n = std::max(x.mag.size(), y.mag.size());
    r.mag.assign(n + 2, 0);
    if (sa == 0 || sb == 0 || sa == sb) {
      const uint64_t mx = sa ? ma : 0, my = sb ? mb : 0;
      u128 carry = 0;
      for (size_t i = 0; i < n; i++) {
        const u128 t = (u128)(i < x.mag.size() ? x.mag[i] : 0) * mx +
                       (u128)(i < y.mag.size() ? y.mag[i] : 0) * my + carry;
        r.mag[i] = (uint64_t)t;
        carry = t >> 64;
      }
      r.mag[n] = (uint64_t)carry;
      r.mag[n + 1] = (uint64_t)(carry >> 64);
      r.sign = sa ? sa : sb;
    } else {
      // |a| |x| - |b| |y| in two's complement, then the sign of sa applied
      __int128 carry = 0;
      for (size_t i = 0; i < n; i++) {
        const __int128 t = (__int128)((u128)(i < x.mag.size() ? x.mag[i] : 0) * ma) -
                           (__int128)((u128)(i < y.mag.size() ? y.mag[i] : 0) * mb) + carry;
        r.mag[i] = (uint64_t)t;
        carry = t >> 64;                            // arithmetic shift
      }
      r.mag[n] = (uint64_t)carry;
      const bool neg = carry < 0;
      r.mag[n + 1] = neg ? ~(uint64_t)0 : 0;
      if (neg) {                                    // magnitude of a negative value
        uint64_t c = 1;
        for (size_t i = 0; i < n + 2; i++) {
          const u128 t = (u128)(~r.mag[i]) + c;
          r.mag[i] = (uint64_t)t;
          c = (uint64_t)(t >> 64);
        }
      }
      r.sign = neg ? -sa : sa;
    }
    r.trim();
    return r;
  }
  // |this| mod m (m > 0), result in [0, m)
  uint64_t mod_small_mag(uint64_t m) const {
    u128 r = 0;
    for (size_t i = mag.size(); i-- > 0;) r = ((r << 64) | mag[i]) % m;
    return (uint64_t)r;
  }
  // this mod m in [0, m)
  uint64_t mod_small(uint64_t m) const {
    uint64_t r = mod_small_mag(m);
    if (sign < 0 && r) r = m - r;
    return r;
  }
  int cmp(const BigInt& b) const {
    if (sign != b.sign) return sign < b.sign ? -1 : 1;
    int c = cmp_mag(mag, b.mag);
    return sign >= 0 ? c : -c;
  }
  int cmp_abs(const BigInt& b) const { return cmp_mag(mag, b.mag); }

  BigInt shl(int64_t bits) const {
    if (sign == 0 || bits == 0) return *this;
    BigInt r;
    r.sign = sign;
    size_t w = (size_t)(bits / 64);
    int s = (int)(bits % 64);
    r.mag.assign(mag.size() + w + 1, 0);
    for (size_t i = 0; i < mag.size(); i++) {
      r.mag[i + w] |= mag[i] << s;
      if (s) r.mag[i + w + 1] |= mag[i] >> (64 - s);
    }
    r.trim();
    return r;
  }

  // Truncated division of magnitudes: q = |a| / |b|, rem = |a| mod |b|
  // (Knuth's algorithm D on 64-bit limbs with 128-bit intermediates).
  static void divmod_mag(const std::vector<uint64_t>& a, const std::vector<uint64_t>& b,
                         std::vector<uint64_t>& q, std::vector<uint64_t>& rem) {
    if (cmp_mag(a, b) < 0) { q.clear(); rem = a; return; }
    const size_t n = b.size(), m = a.size() - n;
    if (n == 1) {
      q.assign(a.size(), 0);
      u128 r = 0;
      for (size_t i = a.size(); i-- > 0;) {
        u128 cur = (r << 64) | a[i];
        q[i] = (uint64_t)(cur / b[0]);
        r = cur % b[0];
      }
      rem.clear();
      if (r) rem.push_back((uint64_t)r);
      while (!q.empty() && q.back() == 0) q.pop_back();
      return;
    }
    const int s = __builtin_clzll(b.back());
    std::vector<uint64_t> vn(n), un(a.size() + 1);
    for (size_t i = n - 1; i > 0; i--) vn[i] = s ? (b[i] << s) | (b[i - 1] >> (64 - s)) : b[i];
    vn[0] = b[0] << s;
    un[a.size()] = s ? a.back() >> (64 - s) : 0;
    for (size_t i = a.size() - 1; i > 0; i--) un[i] = s ? (a[i] << s) | (a[i - 1] >> (64 - s)) : a[i];
    un[0] = a[0] << s;
    q.assign(m + 1, 0);
    for (size_t jj = m + 1; jj-- > 0;) {
      const size_t j = jj;
      u128 num = ((u128)un[j + n] << 64) | un[j + n - 1];
      u128 qhat = num / vn[n - 1];
      u128 rhat = num % vn[n - 1];
      while ((qhat >> 64) != 0 || qhat * vn[n - 2] > ((rhat << 64) | un[j + n - 2])) {
        qhat--;
        rhat += vn[n - 1];
        if ((rhat >> 64) != 0) break;
      }
      // multiply and subtract
      uint64_t borrow = 0, carry = 0;
      for (size_t i = 0; i < n; i++) {
        u128 p = qhat * vn[i] + carry;
        carry = (uint64_t)(p >> 64);
        uint64_t plo = (uint64_t)p;
        u128 d = (u128)un[i + j] - plo - borrow;
        un[i + j] = (uint64_t)d;
        borrow = (uint64_t)(d >> 127);
      }
      u128 d = (u128)un[j + n] - carry - borrow;
      un[j + n] = (uint64_t)d;
      if ((uint64_t)(d >> 127)) {    // went negative: add back once
        qhat--;
        uint64_t c = 0;
        for (size_t i = 0; i < n; i++) {
          u128 t = (u128)un[i + j] + vn[i] + c;
          un[i + j] = (uint64_t)t;
          c = (uint64_t)(t >> 64);
        }
        un[j + n] += c;
      }
      q[j] = (uint64_t)qhat;
    }
    rem.assign(n, 0);
    for (size_t i = 0; i < n; i++) rem[i] = s ? (un[i] >> s) | (un[i + 1] << (64 - s)) : un[i];
    while (!q.empty() && q.back() == 0) q.pop_back();
    while (!rem.empty() && rem.back() == 0) rem.pop_back();
  }
  // Floor division for b > 0 (quotient rounded toward -inf, remainder in [0, b)).
  static void divmod_floor(const BigInt& a, const BigInt& b, BigInt& q, BigInt& r) {
    BigInt qq, rr;
    divmod_mag(a.mag, b.mag, qq.mag, rr.mag);
    qq.sign = qq.mag.empty() ? 0 : a.sign * b.sign;
    rr.sign = rr.mag.empty() ? 0 : a.sign;
    if (rr.sign < 0) {   // a < 0: shift to a non-negative remainder
      qq = qq - from_i64(1);
      rr = rr + b;
    }
    q = qq;
    r = rr;
  }
  static BigInt gcd(BigInt a, BigInt b) {
    a.sign = a.mag.empty() ? 0 : 1;
    b.sign = b.mag.empty() ? 0 : 1;
    while (!b.is_zero()) {
      BigInt q, r;
      divmod_mag(a.mag, b.mag, q.mag, r.mag);
      r.sign = r.mag.empty() ? 0 : 1;
      a = b;
      b = r;
    }
    return a;
  }
  // Exact division (b must divide a).
  static BigInt div_exact(const BigInt& a, const BigInt& b) {
    BigInt q, r;
    divmod_mag(a.mag, b.mag, q.mag, r.mag);
    q.sign = q.mag.empty() ? 0 : a.sign * b.sign;
    return q;
  }
  // little-endian base-2^32 limbs of |this|
  std::vector<uint32_t> limbs32() const {
    std::vector<uint32_t> o;
    for (uint64_t w : mag) { o.push_back((uint32_t)w); o.push_back((uint32_t)(w >> 32)); }
    while (!o.empty() && o.back() == 0) o.pop_back();
    return o;
  }
  static BigInt from_limbs32(const uint32_t* l, size_t n, int sgn) {
    BigInt r;
    for (size_t i = 0; i < n; i += 2) r.mag.push_back((uint64_t)l[i] | (i + 1 < n ? (uint64_t)l[i + 1] << 32 : 0));
    r.sign = sgn;
    r.trim();
    if (!r.mag.empty() && sgn == 0) r.sign = 1;
    return r;
  }
};

}  // namespace dethost

// Host computation of the modular product's parameters.  See crt.hpp.
#include "crt.hpp"

#include <cstring>

namespace cosma {

namespace {

constexpr int32_t kModuli[CRT_MAX_MODULI] = {256, 255, 253, 251, 247, 241, 239, 233,
                                             229, 227, 223, 217, 211, 199, 197, 193};

typedef unsigned __int128 u128;

int floor_log2(u128 x) {
  int b = -1;
  while (x) {
    x >>= 1;
    ++b;
  }
  return b;
}

int ceil_log2(int64_t k) {
  int b = 0;
  while (((int64_t)1 << b) < k) ++b;
  return b;
}

// x^-1 mod p for gcd(x, p) = 1 (extended Euclid).
int32_t inverse_mod(int64_t x, int64_t p) {
  int64_t a = x % p, b = p, u = 1, v = 0;
  while (b) {
    const int64_t q = a / b;
    int64_t t = a - q * b;
    a = b;
    b = t;
    t = u - q * v;
    u = v;
    v = t;
  }
  u %= p;
  if (u < 0) u += p;
  return (int32_t)u;
}

// x in base-2^30 limbs (x < 2^150).
void limbs(u128 x, double* out, int n) {
  const u128 mask = ((u128)1 << CRT_LIMB_BITS) - 1;
  for (int i = 0; i < n; ++i) {
    out[i] = (double)(uint64_t)(x & mask);
    x >>= CRT_LIMB_BITS;
  }
}

}  // namespace

const int32_t* crt_moduli_table() { return kModuli; }

bool crt_params(int64_t k, int nmod, CrtParams* out) {
  if (!out || k < 1 || nmod < CRT_MIN_MODULI || nmod > CRT_MAX_MODULI) return false;
  std::memset(out, 0, sizeof(*out));
  u128 M = 1;
  for (int l = 0; l < nmod; ++l) M *= (u128)kModuli[l];
  const int room = floor_log2(M) - 2 - ceil_log2(k);  // bits for 2 beta
  if (room < 2) return false;                          // beta >= 1
  const int beta = room / 2 < CRT_MAX_BETA ? room / 2 : CRT_MAX_BETA;
  out->nmod = nmod;
  out->beta = beta;
  out->limbs = (floor_log2(M) + CRT_LIMB_BITS) / CRT_LIMB_BITS;
  for (int l = 0; l < nmod; ++l) {
    const int64_t p = kModuli[l];
    const u128 W = M / (u128)p;
    const int32_t inv = inverse_mod((int64_t)(W % (u128)p), p);
    out->p[l] = (int32_t)p;
    out->inv[l] = inv;
    out->pinv[l] = 1.0 / (double)p;
    // (W * inv) mod M by double-and-add over the 9 bits of inv: every
    // intermediate stays below 2 M < 2^127
    u128 T = 0;
    for (int b = 8; b >= 0; --b) {
      T = (T * 2) % M;
      if ((inv >> b) & 1) T = (T + W) % M;
    }
    limbs(T, out->t[l], out->limbs);
  }
  limbs(M, out->mlimb, out->limbs);
  double m = 0.0;
  for (int i = out->limbs - 1; i >= 0; --i) m = m * 0x1p30 + out->mlimb[i];
  out->m_inv = 1.0 / m;
  return true;
}

}  // namespace cosma

// Parameters of the modular (Ozaki scheme II) product: pairwise coprime
// moduli p_l <= 256, their product M, the Chinese-remainder weights M / p_l
// and the operand scale beta.  Computed on the host (exact 128-bit integer
// arithmetic) and passed to the kernels by value.
#pragma once

#include <stdint.h>

#include "tiles.hpp"

namespace cosma {

constexpr int CRT_MAX_MODULI = 16;
constexpr int CRT_MIN_MODULI = 2;
constexpr int CRT_DEFAULT_MODULI = 14;
constexpr int CRT_MAX_BETA = 50;  // residues are taken in binary64 (see ozaki2.hip)

constexpr int CRT_LIMB_BITS = 30;
constexpr int CRT_MAX_LIMBS = 5;  // M < 2^126 for 16 moduli

struct CrtParams {
  int32_t nmod;                      // moduli in use (a prefix of the table)
  int32_t beta;                      // scaled operands satisfy |x| <= 2^beta
  int32_t limbs;                     // 30-bit limbs that hold M (4 or 5)
  int32_t p[CRT_MAX_MODULI];         // moduli
  int32_t inv[CRT_MAX_MODULI];       // (M / p_l)^-1 mod p_l
  double pinv[CRT_MAX_MODULI];       // 1 / p_l rounded to binary64
  // T_l = (M / p_l) * inv_l mod M: T_l = 1 (mod p_l), T_l = 0 (mod p_j, j != l),
  // so X = sum_l r_l T_l = C' (mod M) for residues r_l = C' (mod p_l).
  // Limb i holds bits [30 i, 30 i + 30).
  double t[CRT_MAX_MODULI][CRT_MAX_LIMBS];
  double mlimb[CRT_MAX_LIMBS];       // M in the same limbs
  double m_inv;                      // 1 / M rounded to binary64
};

// Residue planes of the modular path hold, per row tile of `tile` rows (or
// columns of B), kp / 64 contiguous blocks of tile x 64 bytes (one k round
// each); consecutive tiles start CRT_TILE_PAD bytes beyond the end of the
// previous tile's blocks, so that tiles working on the same round at the
// same time do not map onto the same memory channels.
constexpr int64_t CRT_TILE_PAD = 1024;
COSMA_HD inline int64_t crt_tile_stride(int tile, int64_t kp) { return kp * tile + CRT_TILE_PAD; }
COSMA_HD inline int64_t crt_plane_bytes(int64_t extent_padded, int tile, int64_t kp) {
  return extent_padded / tile * crt_tile_stride(tile, kp);
}

// The moduli table: the pairwise coprime integers taken greedily from 256
// downwards.  Exposed for the C ABI.
const int32_t* crt_moduli_table();

// Fill `out` for a reduction length k and nmod moduli.  beta is the largest
// integer with 2 beta + ceil(log2 k) + 2 <= floor(log2 M) (so that every
// |sum_t A'_it B'_tj| <= k 2^(2 beta) <= M / 4), capped at CRT_MAX_BETA.
// Returns false for nmod outside [CRT_MIN_MODULI, CRT_MAX_MODULI], k < 1,
// or when no beta >= 1 exists.
bool crt_params(int64_t k, int nmod, CrtParams* out);

}  // namespace cosma

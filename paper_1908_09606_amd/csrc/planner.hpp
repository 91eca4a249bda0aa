// Host schedule planner: Algorithm 1's FindSeqSchedule, ParallelizeSched and
// FitRanks mapped onto the compute units of one GPU.  Host-only C++17.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/cosma_mi355.h"
#include "tiles.hpp"

namespace cosma {

// Default figures for MI355X (gfx950), used when no device is present.
cosma_device_facts mi355x_defaults();

// Tile menu for a dtype (nullptr / 0 for an unknown dtype).
const TileDesc* tile_menu(int dtype, int* count);

// Bytes per stored operand element, per partial-result element, and the
// MFMA rate per CU per clock in useful flops (2 per multiply-add of the
// product being emulated).
int word_bytes(int dtype);
int partial_bytes(int dtype);
double useful_flops_per_clk_per_cu(int dtype, int slices);

// Slice counts forced through COSMA_OZAKI_SLICES, COSMA_OZAKI_BF16_SLICES and
// COSMA_OZAKI2_MODULI (-1 when unset: the planner chooses from k).
int ozaki_slices();
int ozaki_bf16_slices();
int ozaki2_moduli();

// Error contract of the Ozaki paths (see planner.cpp): bound per unit
// |alpha| k 2^(e_i + f_j) from the emulation, bound per unit D_ij from
// binary64 rounding, and the largest spread k 2^(e_i + f_j) |alpha| / D_ij
// for which the normalised error stays within 3k 2^-53 of the exact product.
struct OzakiBound {
  double scaled;
  double rounding;
  double spread_limit;
};
OzakiBound ozaki_bound(int dtype, int slices, int64_t k, int64_t k_split, int64_t p_k);
// Smallest slice / moduli count whose spread limit reaches `target` (else
// the smallest count with the smallest err_scaled: the most accurate
// emulation); 0 for other dtypes.
int ozaki_choose_slices(int dtype, int64_t k, double target);
// Spread the planner's choice must cover: cosma_set_ozaki_spread, else
// COSMA_OZAKI_SPREAD, else kDefaultOzakiSpread.
constexpr double kDefaultOzakiSpread = 2048.0;
double ozaki_target_spread();
bool set_ozaki_target_spread(double v);
// Fill a plan's err_scaled / err_rounding / spread_limit from its dtype,
// slices, k, k_split and p_k (zeros for the native dtypes).
void set_error_contract(cosma_plan_info* p);
// Largest reduction length per work item of the modular path (int32 sums
// of int8 residue products stay exact).
constexpr int64_t OZAKI2_MAX_K_ITEM = 65536;

// ---- the paper's schedule functions -----------------------------------
double thm1_bound(double m, double n, double k, double S);                 // Theorem 1
void seq_schedule(int64_t S, int64_t* a, int64_t* b);                      // section 5
void par_schedule(double m, double n, double k, double p, double S, double* a, double* b);
double thm2_bound(double m, double n, double k, double p, double S);       // Theorem 2
bool fit_ranks(int64_t m, int64_t n, int64_t k, int64_t p, double delta, int64_t grid[3],
               int64_t* used);                                              // section 7.1
double io_count(int64_t m, int64_t n, int64_t k, int64_t tm, int64_t tn, int64_t kc, int64_t pk,
                bool beta_nonzero);

// Predicted L2 <-> memory traffic (bytes) of a launch that runs `items`
// work items in the xcd_remap / item_coord order, waves of resident slots
// sharing each XCD's L2 (section 5's schedule applied one memory level up).
double q_ea_bytes(int64_t m, int64_t n, int64_t k, int64_t k_split, int64_t splits, int tm,
                  int tn, int group_m, int64_t slots_per_xcd, int num_xcds, double w_bytes);

// Modelled time of one problem inside a persistent batch with a given tile.
double batch_item_cost(int64_t m, int64_t n, int64_t k, int dtype, int tile_id,
                       const cosma_device_facts& f);

// Device workspace a plan needs (split-K partials, Ozaki digit planes).
size_t workspace_bytes(const cosma_plan_info& p);

// ---- GPU plan -----------------------------------------------------------
// Fill `out` for a given tile and split (tile_id < 0 / p_k <= 0: planner's
// choice).  Returns a cosma_status.
// a_pitch_bytes: A's row pitch (lda * element size); 0 means dense (k).
int make_plan(int64_t m, int64_t n, int64_t k, int dtype, const cosma_device_facts& f,
              double delta, int tile_id, int p_k, cosma_plan_info* out,
              int64_t a_pitch_bytes = 0);

// True when rows of A at the same k offset fall into the same L2 sets: a row
// pitch that is a multiple of 4 KiB.
bool conflicting_pitch(int64_t a_pitch_bytes);

}  // namespace cosma

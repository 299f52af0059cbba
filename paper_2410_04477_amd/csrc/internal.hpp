// Internal interfaces between the C ABI layer and the kernels.
#pragma once

#include "common.hpp"

namespace bv {

struct FwdArgs {
  const double* locs;
  const double* y;
  const int* block_ptr;
  const int* nbr_ptr;
  const int* nbr_idx;
  const int* sched;      // block ids of this size class (schedule mode)
  const int* list;       // (theta, block) pairs, packed theta * bc + block (list mode)
  const int* list_count; // device count of list entries (list mode)
  int nsched;            // schedule mode: blocks in this class
  int ntheta;
  int bc;
  int d;
  int fp32_guard;        // 1: flag blocks whose FP32 pivots fall below the guard
  int flag_or;           // OR-ed into every flag written (4 marks an FP64 re-factorisation)
  double* partial;       // [theta * bc + block]
  int* flag;             // [theta * bc + block]: 1 guard tripped, 2 non-positive pivot, 4 re-run in FP64
};

hipError_t launch_forward(int cfg, bool fp32, const FwdArgs& a, const ThetaPack& thp, int grid, hipStream_t s);

struct AdjArgs {
  const double* locs;
  const double* y;
  const int* block_ptr;
  const int* nbr_ptr;
  const int* nbr_idx;
  const int* sched;
  const int* list;
  const int* list_count;
  int nsched;
  int ntheta;
  int bc;
  int d;
  int fp32_guard;
  int flag_or;
  int ldx;               // leading dimension of the LDS right-hand sides (>= l_max + 2)
  double* partial;       // [theta * bc + block]
  double* gpart;         // [(theta * bc + block) * 3 + k]
  int* flag;
  double* coef;          // coefficient mode: conditional-mean weights, CSR like nbr_idx, one copy per theta
  double* cvar;          // coefficient mode: conditional variance per block and theta
  int64_t coef_stride;   // coefficient mode: entries per theta (nbr_ptr[bc])
  void* tiles;           // one-wave adjoint: factor tiles, one slot per work item of the launch
  int item_base;         // first work item of the launch (launches in chunks of the tile buffer)
  // prediction (one-wave mode 4): block rows come from locs2 (new locations in
  // block order), neighbour rows from locs / y (observations)
  const double* locs2;
  double* out_mean;      // [new location]: conditional mean
  double* out_var;       // [new location]: conditional variance
  double* out_cov;       // [block][ldc][ldc]: conditional covariance, or null
  int ldc;
  int gen;               // some theta of the launch has nu outside {1/2, 3/2, 5/2} (Bessel form)
  double* gnu;           // Bessel-form gradient launches: d l_i / d nu [theta * bc + block], or null
};

hipError_t launch_adjoint(int cfg, bool fp32, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s);
size_t adjoint_lds_need(int cfg, bool fp32, int ldx);   // LDS bytes of one launch
hipError_t launch_coefficients(int cfg, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s);
// matrix-core engine: g tile rows (1..11); mode 0 value, 1 value + gradient, 2 coefficients (FP64)
hipError_t launch_mfma(int g, bool fp32, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s);
size_t mfma_lds_need(int g, bool fp32, int mode, int ldx);   // dynamic LDS bytes of one launch
// one-wave matrix-core kernels (mode 0 value, 1 value + gradient); FP32 up to
// G = kWaveMaxG32 tile rows, FP64 up to kWaveMaxG64 (above G = 8 the FP64 tiles
// exceed the register file and part of them spills to scratch)
constexpr int kWaveMaxG32 = 11;
constexpr int kWaveMaxG64 = 11;
constexpr int kWaveChunk = 32;  // adjoint right-hand sides per pass, at most (bounds the LDS of any block)
// right-hand sides per pass of a class with g tile rows: 28 up to g = 9, which
// keeps the one-wave adjoint's LDS at or under 20 kB (eight waves per CU)
__host__ __device__ constexpr int wave_chunk(int g) { return g <= 9 ? 28 : kWaveChunk; }
// bytes of one work item's slot in the adjoint's tile buffer (factor tiles and
// the border row), and the buffer's cap
inline size_t wave_tile_bytes(int g, bool fp32) { return ((size_t)g * (g + 1) / 2 * 256 + 16 * (size_t)g) * (fp32 ? 4 : 8); }
constexpr size_t kAdjTileCap = (size_t)4 << 30;
bool wave_fits(int g, bool fp32);
// gradient as two launches (factor + tiles, then the adjoint from the tiles)
inline bool wave_split(int g, bool fp32) { return fp32 && g >= 10; }
// FP64 classes above G = 9: the factor + tiles launch left-looking by tile
// columns (one tile column in the registers at a time), then the adjoint launch
inline bool wave_left(int g, bool fp32) { return !fp32 && g >= 10; }
// gradient in one launch with the factor kept in the registers (no tile
// buffer): FP64 classes up to G = 9, FP32 up to G = 10 (two waves per SIMD up
// to G = 9, one at G = 10, which still beats the split gradient there: 315
// against 307 evals/s at n = 1e6).  The right-hand sides go in passes of
// wave_chunk(G), except at G = 9, where the registers the pass loop holds
// would spill: there only classes whose l_max + 2 right-hand sides fit one pass
#ifndef BV_REGADJ_MAX_G32
#define BV_REGADJ_MAX_G32 10
#endif
#ifndef BV_REGADJ_MAX_G64
#define BV_REGADJ_MAX_G64 9
#endif
__host__ __device__ constexpr bool wave_regadj_passes(int g, bool /*fp32*/) { return g != 9; }
inline bool wave_regadj(int g, bool fp32, int lmax) {
  return g >= 1 && g <= (fp32 ? BV_REGADJ_MAX_G32 : BV_REGADJ_MAX_G64) &&
         (wave_regadj_passes(g, fp32) || lmax + 2 <= wave_chunk(g));
}
// prediction: round the conditioning-set size up to the factorisation's panel width
__host__ __device__ constexpr int pred_rows(int m) { return (m + 3) & ~3; }
hipError_t launch_wave_f32(int g, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s);
hipError_t launch_wave_f64(int g, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s);
hipError_t launch_wave_gen_f32(int g, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s);
hipError_t launch_wave_gen_f64(int g, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s);
// dispatches on a.gen to the closed-form or the Bessel-form kernels
hipError_t launch_wave(int g, bool fp32, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s);
struct LargeArgs {
  const double* locs;
  const double* y;
  const int* block_ptr;
  const int* nbr_ptr;
  const int* nbr_idx;
  const int* sched;
  const int* list;
  const int* list_count;
  int nsched;
  int ntheta;
  int bc;
  int d;
  int fp32_guard;
  int flag_or;
  void* ws;              // nslots x slot_elems elements
  int64_t slot_elems;    // large_slot_elems(p_max, l_max)
  double* partial;
  int* flag;
  double* gpart;         // gradient launches: [(theta * bc + block) * 3 + k]
};
constexpr int kLargeCfg = 31;   // size class of blocks above the register capacity
// bytes of large-block slots above which a plan factors no more than 256 blocks at a time
constexpr size_t kLargeSlotCap = (size_t)4 << 30;
// elements of one large-block slot: the P x P matrix, the gradient's P x 16 ceil((l + 2) / 16)
// right-hand sides and 3 P staged coordinates, P = 16 ceil((p_max + 1) / 16)
size_t large_slot_elems(int pmax, int lmax);
hipError_t launch_large(bool fp32, bool grad, const LargeArgs& a, const ThetaPack& thp, int grid, hipStream_t s);

// leading dimension of the LDS right-hand sides for l_max (matrix-core engine)
inline int mfma_ldx(int nr_max) { return 16 * ((nr_max + 15) / 16) + 1; }

// mpad: conditioning-set sizes are rounded up to a multiple of mpad (4 for
// prediction plans, whose neighbour rows end on a panel boundary)
hipError_t launch_classify(const int* block_ptr, const int* nbr_ptr, int bc, int* cfg_of, int* counts,
                           unsigned long long* stats, int* maxes, int* lmax_cfg, int engine, int mpad,
                           hipStream_t s);
hipError_t launch_scatter(const int* cfg_of, int bc, const int* cfg_off, int* cursor, int* sched, hipStream_t s);
hipError_t launch_remap(int* cfg_of, int bc, const int* remap, hipStream_t s);
// size classes with fewer blocks than this run with the next larger populated class
constexpr int kMergeBelow = 256;
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s);
hipError_t launch_compact_flagged(const int* sched, int nsched, int ntheta, int bc, const int* flag, int* list,
                                  int* count, hipStream_t s);
hipError_t launch_reduce_partials(const double* partial, const int* flag, int bc, int ntheta, int fp64_only,
                                  double* out, int* counters, hipStream_t s);
hipError_t launch_reduce_vec(const double* vec, int bc, int k, int ntheta, double* out, hipStream_t s);

// Per-call device buffers of the value path (the plan's workspace, or the
// static array of vecchia_loglik_noalloc): partial and flag hold
// ntheta * bc entries, list ntheta * bc, count one per size class.
struct CallBuffers {
  double* partial;
  int* flag;
  int* list;
  int* count;
};
// Argument checks of vecchia_loglik (need_aux: the plan's auxiliary workspace
// must be attached when it has one).
int check_loglik_args(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                      const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                      const vecchia_theta* theta, int32_t ntheta, int32_t precision, const double* loglik,
                      bool need_aux);
int loglik_run(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
               const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
               const vecchia_theta* theta, int32_t ntheta, int32_t precision, double* loglik,
               int32_t* counters, double* partial, const CallBuffers& cb, void* stream);
// Resolves, once per device, the device address of the static array behind
// vecchia_loglik_noalloc, for the current device.
int noalloc_prepare_current_device();

}  // namespace bv

// C ABI of the block Vecchia library: argument checking, workspace layout,
// launch orchestration.  Every numerical step runs in the HIP kernels.
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "internal.hpp"

using namespace bv;

#define VCHECK_HIP(x)                        \
  do {                                       \
    hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) return VECCHIA_EHIP; \
  } while (0)

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" int vecchia_version(void) { return 10000; }

extern "C" int32_t vecchia_plan_layout(int64_t* out, int32_t cap) {
#define BV_OFF(f) (int64_t) offsetof(vecchia_plan, f)
  const int64_t v[] = {(int64_t)sizeof(vecchia_plan), BV_OFF(n), BV_OFF(bc), BV_OFF(max_theta), BV_OFF(nbuckets),
                       BV_OFF(pmax), BV_OFF(lmax), BV_OFF(mmax), BV_OFF(bucket_cfg), BV_OFF(bucket_off),
                       BV_OFF(lsum), BV_OFF(flops_la), BV_OFF(cov_entries), BV_OFF(ws), BV_OFF(ws_bytes),
                       BV_OFF(off_sched), BV_OFF(off_partial), BV_OFF(off_flag), BV_OFF(off_list),
                       BV_OFF(off_count), BV_OFF(off_chunk), BV_OFF(off_grad), BV_OFF(timing), BV_OFF(engine),
                       BV_OFF(nlarge), BV_OFF(large_slots), BV_OFF(large_slot_elems), BV_OFF(aux_ws_bytes),
                       BV_OFF(aux_ws), BV_OFF(bucket_lmax), BV_OFF(lds_bytes), BV_OFF(bucket_main), BV_OFF(exec),
                       BV_OFF(kind)};
#undef BV_OFF
  const int32_t k = (int32_t)(sizeof(v) / sizeof(v[0]));
  if (out)
    for (int32_t i = 0; i < k && i < cap; ++i) out[i] = v[i];
  return k;
}

extern "C" const char* vecchia_status_string(int status) {
  switch (status) {
    case VECCHIA_OK: return "ok";
    case VECCHIA_EINVAL: return "invalid argument";
    case VECCHIA_ENOMEM: return "workspace or output capacity too small";
    case VECCHIA_EHIP: return "HIP runtime error";
    case VECCHIA_EUNSUPPORTED: return "unsupported input";
    default: return "unknown status";
  }
}

// ---------------------------------------------------------------- plan ----

namespace {
struct PlanLayout {
  size_t sched, partial, flag, list, count, chunk, grad, scratch, total;
};

PlanLayout plan_layout(int64_t bc, int32_t max_theta) {
  PlanLayout L;
  size_t o = 0;
  const size_t nb = (size_t)bc, nt = (size_t)max_theta;
  L.sched = o;   o = align256(o + sizeof(int) * nb);
  L.partial = o; o = align256(o + sizeof(double) * nb * nt);
  L.flag = o;    o = align256(o + sizeof(int) * nb * nt);
  L.list = o;    o = align256(o + sizeof(int) * nb * nt);
  L.count = o;   o = align256(o + sizeof(int) * 64);
  L.chunk = o;   o = align256(o + sizeof(double) * 64);
  L.grad = o;    o = align256(o + sizeof(double) * nb * nt * 4);   // 3 per block, then d/d nu per block
  L.scratch = o; o = align256(o + sizeof(int) * (nb + 256) + sizeof(unsigned long long) * 8);
  L.total = o;
  return L;
}

// Digamma psi(x) for x > 0: the recurrence psi(x) = psi(x + 1) - 1/x up to
// x >= 8, then the asymptotic series psi(x) ~ log x - 1/(2x) - sum_k
// B_2k / (2k x^2k) (Abramowitz and Stegun 6.3.18) to the x^-14 term, whose
// first omitted term is below 1e-17 there.
static double digamma(double x) {
  double acc = 0.0;
  while (x < 8.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  const double r = 1.0 / (x * x);
  // B_2k / (2k): 1/12, -1/120, 1/252, -1/240, 1/132, -691/32760, 1/12
  const double series =
      r * (1.0 / 12 - r * (1.0 / 120 - r * (1.0 / 252 - r * (1.0 / 240 - r * (1.0 / 132 - r * (691.0 / 32760 - r / 12))))));
  return acc + log(x) - 0.5 / x - series;
}

// Orders of the Bessel form: nu in [kNuMin, kNuMax] (outside the closed forms).
constexpr double kNuMin = 0.05, kNuMax = 10.0;

// VECCHIA_OK, VECCHIA_EINVAL (bad value) or VECCHIA_EUNSUPPORTED (nu outside
// what the kernels evaluate).
int theta_status(const vecchia_theta& t, int d, ThetaDev& o) {
  memset(&o, 0, sizeof(o));
  if (!(t.sigma2 > 0) || !(t.range > 0) || !(t.nugget >= 0) || !isfinite(t.sigma2) || !isfinite(t.range) ||
      !isfinite(t.nugget) || !(t.nu > 0) || !isfinite(t.nu))
    return VECCHIA_EINVAL;
  if (!(t.nu >= kNuMin && t.nu <= kNuMax)) return VECCHIA_EUNSUPPORTED;
  o.nu_code = t.nu == 0.5 ? 0 : t.nu == 1.5 ? 1 : t.nu == 2.5 ? 2 : 3;
  {
    // order-only constants of the Bessel form, also for the closed-form orders
    // (a launch that holds any other nu evaluates all its thetas that way):
    // nu = n + mu with |mu| <= 1/2; for small mu, Gamma1 from the Taylor series
    // of 1/Gamma(1 + z) (Abramowitz and Stegun 6.1.34), which avoids the
    // cancellation of the difference quotient
    BesselOrder& b = o.bes;
    b.n = (int)floor(t.nu + 0.5);
    const double mu = t.nu - b.n;
    b.mu = mu;
    b.gplus = tgamma(1.0 + mu);
    b.gminus = tgamma(1.0 - mu);
    const double rp = 1.0 / b.gplus, rm = 1.0 / b.gminus;
    b.gam2 = 0.5 * (rm + rp);
    b.gam1 = fabs(mu) < 1e-3 ? -(0.5772156649015329 - 0.0420026350340952 * mu * mu) : (rm - rp) / (2.0 * mu);
    b.mu_pi_csc = fabs(mu) < 1e-14 ? 1.0 : M_PI * mu / sin(M_PI * mu);
    b.lognorm = (1.0 - t.nu) * log(2.0) - lgamma(t.nu);
    b.dlognorm = -log(2.0) - digamma(t.nu);
  }
  o.sigma2 = t.sigma2;
  o.nugget = t.nugget;
  o.inv_range = 1.0 / t.range;
  for (int k = 0; k < 3; ++k) {
    if (k < d) {
      if (!(t.aniso[k] > 0) || !isfinite(t.aniso[k])) return VECCHIA_EINVAL;
      o.inv_scale[k] = 1.0 / (t.range * t.aniso[k]);
    } else {
      o.inv_scale[k] = 0.0;
    }
  }
  return VECCHIA_OK;
}

bool theta_to_dev(const vecchia_theta& t, int d, ThetaDev& o) { return theta_status(t, d, o) == VECCHIA_OK; }

template <typename P> P* at(void* base, size_t off) { return reinterpret_cast<P*>(static_cast<char*>(base) + off); }

// Side streams (default priority) on which the size classes other than the
// largest run concurrently with it; forked from and joined back to the
// caller's stream with events.
constexpr int kSideStreams = 3;
struct Exec {
  hipStream_t side[kSideStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSideStreams] = {};
  hipEvent_t mark = nullptr;   // end of a split class's first factorisation launch
};
}  // namespace

extern "C" int vecchia_tile_config(int32_t engine, int32_t cfg, int32_t* R, int32_t* G) {
  if (!R || !G) return VECCHIA_EINVAL;
  if (engine == kEngineMfma || engine == kEngineMfmaWg) {
    if (cfg < 0 || cfg >= kMfmaMaxG) return VECCHIA_EINVAL;
    *R = 16;
    *G = cfg + 1;
    return VECCHIA_OK;
  }
  if (engine != kEngineTiles || cfg < 0 || cfg >= kNumCfgs) return VECCHIA_EINVAL;
  *R = kCfgs[cfg].R;
  *G = kCfgs[cfg].G;
  return VECCHIA_OK;
}

extern "C" size_t vecchia_plan_workspace_size(int64_t bc, int32_t max_theta) {
  if (bc <= 0 || max_theta <= 0) return 0;
  return plan_layout(bc, max_theta).total;
}

extern "C" int vecchia_plan_init(vecchia_plan* plan, const int32_t* block_ptr, const int32_t* nbr_ptr, int64_t n,
                                 int64_t bc, int32_t max_theta, int32_t engine, void* workspace, size_t ws_bytes,
                                 void* stream) {
  if (!plan || !block_ptr || !nbr_ptr || !workspace || n <= 0 || bc <= 0 || bc > n || max_theta <= 0 ||
      n >= (int64_t)1 << 31 || (int64_t)bc * max_theta >= (int64_t)1 << 31)
    return VECCHIA_EINVAL;
  const bool predict = (engine & VECCHIA_PLAN_PREDICT) != 0;
  engine &= ~VECCHIA_PLAN_PREDICT;
  if (engine != kEngineMfma && engine != kEngineTiles && engine != kEngineMfmaWg) return VECCHIA_EINVAL;
  if (predict && (engine != kEngineMfma || max_theta != 1)) return VECCHIA_EINVAL;
  const PlanLayout L = plan_layout(bc, max_theta);
  if (ws_bytes < L.total) return VECCHIA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  memset(plan, 0, sizeof(*plan));  // a plan with timing enabled must disable it before re-initialisation
  int* cfg_of = at<int>(workspace, L.scratch);
  int* counts = at<int>(workspace, L.count);            // [0..32) counts, [32..64) cursors/offsets
  unsigned long long* stats = at<unsigned long long>(workspace, L.chunk);
  int* maxes = at<int>(workspace, L.chunk + 128);
  int* lmax_cfg = at<int>(workspace, L.chunk + 256);    // [0..32) largest l_i per configuration
  VCHECK_HIP(launch_fill_int(counts, 64, 0, s));
  VCHECK_HIP(launch_fill_int(maxes, 16, 0, s));
  VCHECK_HIP(launch_fill_int(lmax_cfg, 32, 0, s));
  VCHECK_HIP(launch_fill_int(reinterpret_cast<int*>(stats), 16, 0, s));
  VCHECK_HIP(launch_classify(block_ptr, nbr_ptr, (int)bc, cfg_of, counts, stats, maxes, lmax_cfg, engine,
                             predict ? 4 : 1, s));
  int hcounts[32];
  int hmax[4];
  int hlmax[32];
  unsigned long long hstats[4];
  VCHECK_HIP(hipMemcpyAsync(hcounts, counts, sizeof(hcounts), hipMemcpyDeviceToHost, s));
  VCHECK_HIP(hipMemcpyAsync(hmax, maxes, sizeof(hmax), hipMemcpyDeviceToHost, s));
  VCHECK_HIP(hipMemcpyAsync(hlmax, lmax_cfg, sizeof(hlmax), hipMemcpyDeviceToHost, s));
  VCHECK_HIP(hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, s));
  VCHECK_HIP(hipStreamSynchronize(s));
  if (hmax[3] > 0) {
    // a block with no points, or larger than even the global-workspace kernel takes
    return hmax[0] > 16383 ? VECCHIA_EUNSUPPORTED : VECCHIA_EINVAL;
  }
  // prediction has no large-block path: every block must fit the one-wave kernel
  if (predict && hcounts[kLargeCfg] > 0) return VECCHIA_EUNSUPPORTED;
  const int ncfg = engine == kEngineTiles ? kNumCfgs : kMfmaMaxG;
  // merge sparse size classes upward: a class's kernel also takes every smaller
  // block, and a launch of a few blocks costs a whole block's latency
  int remap[32];
  for (int c = 0; c < 32; ++c) remap[c] = c;
  bool merged = false;
  for (int c = 0; c < ncfg; ++c) {
    if (hcounts[c] <= 0 || hcounts[c] >= kMergeBelow) continue;
    int c2 = c + 1;
    while (c2 < ncfg && hcounts[c2] == 0) ++c2;
    if (c2 >= ncfg) continue;
    hcounts[c2] += hcounts[c];
    hlmax[c2] = hlmax[c2] > hlmax[c] ? hlmax[c2] : hlmax[c];
    hcounts[c] = 0;
    for (int c0 = 0; c0 <= c; ++c0)
      if (remap[c0] == c) remap[c0] = c2;
    merged = true;
  }
  if (merged) {
    int* remap_d = at<int>(workspace, L.chunk + 384);
    VCHECK_HIP(hipMemcpyAsync(remap_d, remap, sizeof(remap), hipMemcpyHostToDevice, s));
    VCHECK_HIP(launch_remap(cfg_of, (int)bc, remap_d, s));
  }
  int hoff[32] = {0};
  int acc = 0, nb = 0;
  for (int c = 0; c < ncfg; ++c) {
    hoff[c] = acc;
    if (hcounts[c] > 0) {
      plan->bucket_cfg[nb] = c;
      plan->bucket_off[nb] = acc;
      plan->bucket_lmax[nb] = hlmax[c];
      ++nb;
    }
    acc += hcounts[c];
  }
  plan->nlarge = hcounts[kLargeCfg];
  if (plan->nlarge > 0) {
    hoff[kLargeCfg] = acc;
    plan->bucket_cfg[nb] = kLargeCfg;
    plan->bucket_off[nb] = acc;
    plan->bucket_lmax[nb] = hlmax[kLargeCfg];
    ++nb;
    acc += hcounts[kLargeCfg];
    const int64_t work = plan->nlarge * (int64_t)max_theta;
    plan->large_slot_elems = (int64_t)large_slot_elems(hmax[0], hlmax[kLargeCfg]);
    // one workgroup per slot: up to 8 per compute unit while the slots fit in
    // kLargeSlotCap bytes, at least one per compute unit
    const int64_t by_mem = (int64_t)(kLargeSlotCap / ((size_t)plan->large_slot_elems * sizeof(double)));
    int64_t slots = by_mem < 2048 ? by_mem : 2048;
    if (slots < 256) slots = 256;
    plan->large_slots = (int32_t)(work < slots ? work : slots);
    plan->aux_ws_bytes = (size_t)plan->large_slots * (size_t)plan->large_slot_elems * sizeof(double);
  }
  if (engine == kEngineMfma && !predict) {
    // adjoint factor tiles, FP64, of every work item of the classes whose
    // gradient goes through the tile buffer (the others keep the factor in
    // registers), so that the classes can run concurrently; capped
    size_t need = 0;
    for (int c = 0; c < kMfmaMaxG; ++c)
      if (hcounts[c] > 0 && wave_fits(c + 1, false) && !wave_regadj(c + 1, false, hlmax[c]))
        need += (size_t)hcounts[c] * (size_t)max_theta * wave_tile_bytes(c + 1, false);
    if (need > kAdjTileCap) need = kAdjTileCap;
    plan->aux_ws_bytes += need;   // the tile buffer follows the large-block slots
  }
  plan->bucket_off[nb] = acc;
  plan->nbuckets = nb;
  VCHECK_HIP(hipMemcpyAsync(counts + 32, hoff, sizeof(int) * 32, hipMemcpyHostToDevice, s));
  VCHECK_HIP(launch_fill_int(counts, 32, 0, s));
  VCHECK_HIP(launch_scatter(cfg_of, (int)bc, counts + 32, counts, at<int>(workspace, L.sched), s));
  VCHECK_HIP(hipStreamSynchronize(s));
  plan->n = n;
  plan->bc = bc;
  plan->max_theta = max_theta;
  plan->pmax = hmax[0];
  plan->lmax = hmax[1];
  plan->mmax = hmax[2];
  plan->flops_la = (double)hstats[0] / 3.0 + (double)hstats[1];
  plan->cov_entries = (double)hstats[2];
  plan->lsum = (int64_t)hstats[3];
  plan->ws = workspace;
  plan->ws_bytes = ws_bytes;
  plan->off_sched = L.sched;
  plan->off_partial = L.partial;
  plan->off_flag = L.flag;
  plan->off_list = L.list;
  plan->off_count = L.count;
  plan->off_chunk = L.chunk;
  plan->off_grad = L.grad;
  plan->engine = engine;
  plan->kind = predict ? 1 : 0;
  // the static array of vecchia_loglik_noalloc: its device address on this
  // device is resolved here, at set-up, rather than inside a later call (a
  // failure is reported by that entry point)
  (void)noalloc_prepare_current_device();
  int dev = 0, lds = 0;
  VCHECK_HIP(hipGetDevice(&dev));
  VCHECK_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  plan->lds_bytes = lds;
  int big = 0;
  for (int q = 1; q < nb; ++q)
    if (plan->bucket_off[q + 1] - plan->bucket_off[q] > plan->bucket_off[big + 1] - plan->bucket_off[big]) big = q;
  plan->bucket_main = big;
  if (nb > 1) {
    Exec* ex = new Exec();
    plan->exec = ex;
    VCHECK_HIP(hipEventCreateWithFlags(&ex->fork, hipEventDisableTiming));
    VCHECK_HIP(hipEventCreateWithFlags(&ex->mark, hipEventDisableTiming));
    for (int k = 0; k < kSideStreams; ++k) {
      VCHECK_HIP(hipStreamCreateWithFlags(&ex->side[k], hipStreamNonBlocking));
      VCHECK_HIP(hipEventCreateWithFlags(&ex->join[k], hipEventDisableTiming));
    }
  }
  return VECCHIA_OK;
}

// Forward arguments in the form the matrix-core kernels take.
static AdjArgs as_adj(const FwdArgs& f, const vecchia_plan* plan) {
  AdjArgs a;
  memset(&a, 0, sizeof(a));
  a.locs = f.locs;
  a.y = f.y;
  a.block_ptr = f.block_ptr;
  a.nbr_ptr = f.nbr_ptr;
  a.nbr_idx = f.nbr_idx;
  a.sched = f.sched;
  a.list = f.list;
  a.list_count = f.list_count;
  a.nsched = f.nsched;
  a.ntheta = f.ntheta;
  a.bc = f.bc;
  a.d = f.d;
  a.fp32_guard = f.fp32_guard;
  a.flag_or = f.flag_or;
  a.ldx = 0;   // set per size class
  a.partial = f.partial;
  a.flag = f.flag;
  return a;
}

// Matrix-core kernel of size class q: the one-wave kernels where the class
// fits them (engine MFMA), else the four-wave kernels.  mode 0: value,
// 1: value + gradient.  VECCHIA_EUNSUPPORTED when the four-wave adjoint's
// right-hand sides do not fit the device LDS.
// One-wave kernel mode that size class q runs for a value (with_grad = 0) or
// value + gradient call: 0 value, 5 gradient with the factor in registers,
// 1 gradient through the tile buffer, 23 the split gradient (mode 2 then 3);
// -1 when the class does not run the one-wave kernels.
// whether the largest class waits for the first factorisation half of the
// split class (one wave per SIMD) before it starts; a build switch, measured
// neutral since FP32 G = 10 moved to the register-resident kernel
#ifndef BV_MARK_SPLIT
#define BV_MARK_SPLIT 1
#endif
constexpr bool kMarkSplit = BV_MARK_SPLIT;
static int class_wave_mode(const vecchia_plan* plan, int q, bool fp32, bool with_grad) {
  const int g = plan->bucket_cfg[q] + 1;
  // (the FP64 one-wave value kernels above G = 9 spill part of their tiles,
  // yet at n = 1e6 they run faster than the four-wave kernels, whose tiles fit;
  // the FP64 gradient there factors left-looking, mode 6, and takes the
  // adjoint from the stored tiles)
  if (plan->engine != kEngineMfma || plan->bucket_cfg[q] == kLargeCfg || !wave_fits(g, fp32)) return -1;
  if (!with_grad) return 0;
  if (wave_regadj(g, fp32, plan->bucket_lmax[q])) return 5;
  if (wave_left(g, fp32)) return 63;
  return wave_split(g, fp32) ? 23 : 1;
}

extern "C" int vecchia_plan_class_kernel(const vecchia_plan* plan, int32_t q, int32_t precision, int32_t with_grad,
                                         char* name, int32_t cap) {
  if (!plan || q < 0 || q >= plan->nbuckets || !name || cap < 1) return VECCHIA_EINVAL;
  const bool fp32 = precision != VECCHIA_FP64;
  const char* t = fp32 ? "float" : "double";
  const int g = plan->bucket_cfg[q] + 1;
  const int mode = class_wave_mode(plan, q, fp32, with_grad != 0);
  int n;
  if (plan->bucket_cfg[q] == kLargeCfg)
    n = snprintf(name, (size_t)cap, "bv_large_kernel<%s>", t);
  else if (mode == 23 || mode == 63)
    n = snprintf(name, (size_t)cap, "bv_wave_kernel<%s,%d,%d>+bv_wave_kernel<%s,%d,3>", t, g, mode / 10, t, g);
  else if (mode >= 0)
    n = snprintf(name, (size_t)cap, "bv_wave_kernel<%s,%d,%d>", t, g, mode);
  else if (plan->engine == kEngineTiles)
    n = snprintf(name, (size_t)cap, "bv_%s_kernel<%s,cfg%d>", with_grad ? "adj" : "fwd", t, plan->bucket_cfg[q]);
  else
    n = snprintf(name, (size_t)cap, "bv_mfma_kernel<%s,%d,%d>", t, g, with_grad ? 1 : 0);
  return n >= 0 && n < cap ? VECCHIA_OK : VECCHIA_ENOMEM;
}

static int launch_mfma_class(const vecchia_plan* plan, int q, bool fp32, int mode, AdjArgs a, const ThetaPack& thp,
                             int grid, hipStream_t s, void* tiles, size_t tile_bytes, hipStream_t s2 = nullptr,
                             hipEvent_t mark = nullptr) {
  const int g = plan->bucket_cfg[q] + 1;
  a.gen = a.gnu != nullptr;   // d / d nu needs the Bessel-form kernels whatever nu is
  for (int t = 0; t < a.ntheta; ++t) a.gen |= thp.t[t].nu_code == 3;
  const int wmode = class_wave_mode(plan, q, fp32, mode != 0);
  if (wmode >= 0) {
    if (mode == 0) {
      VCHECK_HIP(launch_wave(g, fp32, 0, a, thp, grid, s));
      return VECCHIA_OK;
    }
    if (wmode == 5) {   // no tile buffer needed
      VCHECK_HIP(launch_wave(g, fp32, 5, a, thp, grid, s));
      return VECCHIA_OK;
    }
    // adjoint: as many work items per launch as its part of the tile buffer holds
    const size_t per = wave_tile_bytes(g, fp32);
    const size_t cap = tile_bytes / per;
    if (cap == 0) return VECCHIA_ENOMEM;
    const int chunk = cap < (size_t)grid ? (int)cap : grid;
    // two launches: the factorisation + tile store (mode 2, or mode 6 for the
    // FP64 left-looking one; its Bessel-form variant is not built: mode 1
    // there), then the adjoint (mode 3)
    const bool two = wmode == 23 || (wmode == 63 && !a.gen);
    const int fm = wmode == 63 ? 6 : 2;
    if (s2 && two && chunk == grid && grid >= 2) {
      // the split gradient in two halves on two streams: the adjoint launch of
      // one half overlaps the factorisation launch of the other, each half
      // with its own part of the tile buffer
      constexpr int kPieces = 2;
      const int h = (grid + kPieces - 1) / kPieces;
      for (int k = 0; k * h < grid; ++k) {
        a.item_base = k * h;
        a.tiles = static_cast<char*>(tiles) + (size_t)k * h * per;
        const int n = grid - k * h < h ? grid - k * h : h;
        const hipStream_t sk = (k & 1) ? s2 : s;
        VCHECK_HIP(launch_wave(g, fp32, fm, a, thp, n, sk));
        if (k == 0 && mark) VCHECK_HIP(hipEventRecord(mark, sk));
        VCHECK_HIP(launch_wave(g, fp32, 3, a, thp, n, sk));
      }
      return VECCHIA_OK;
    }
    a.tiles = tiles;
    for (int w0 = 0; w0 < grid; w0 += chunk) {
      a.item_base = w0;
      const int n = grid - w0 < chunk ? grid - w0 : chunk;
      if (two) {
        VCHECK_HIP(launch_wave(g, fp32, fm, a, thp, n, s));
        VCHECK_HIP(launch_wave(g, fp32, 3, a, thp, n, s));
      } else {
        VCHECK_HIP(launch_wave(g, fp32, 1, a, thp, n, s));
      }
    }
    return VECCHIA_OK;
  }
  a.ldx = mfma_ldx(plan->bucket_lmax[q] + 2);
  if (mfma_lds_need(g, fp32, mode, a.ldx) > (size_t)plan->lds_bytes) return VECCHIA_EUNSUPPORTED;
  VCHECK_HIP(launch_mfma(g, fp32, mode, a, thp, grid, s));
  return VECCHIA_OK;
}

// Vector-ALU adjoint of size class q (right-hand sides held whole in LDS).
static int launch_tiles_adjoint(const vecchia_plan* plan, int q, bool fp32, AdjArgs a, const ThetaPack& thp,
                                int grid, hipStream_t s) {
  a.ldx = plan->bucket_lmax[q] + 2;
  if (adjoint_lds_need(plan->bucket_cfg[q], fp32, a.ldx) > (size_t)plan->lds_bytes) return VECCHIA_EUNSUPPORTED;
  VCHECK_HIP(launch_adjoint(plan->bucket_cfg[q], fp32, a, thp, grid, s));
  return VECCHIA_OK;
}

#define VCHECK_ST(x)            \
  do {                          \
    int st_ = (x);              \
    if (st_) return st_;        \
  } while (0)

// Stream of size class q: the largest class stays on the caller's stream, the
// others go round-robin to the plan's side streams when `conc`.
static hipStream_t class_stream(const vecchia_plan* plan, int q, hipStream_t s, bool conc) {
  if (!conc || q == plan->bucket_main) return s;
  const int k = (q < plan->bucket_main ? q : q - 1) % kSideStreams;
  return static_cast<Exec*>(plan->exec)->side[k];
}
// A side stream that no size class uses (the last one, when the classes other
// than the largest leave it free), or null.
static hipStream_t spare_stream(const vecchia_plan* plan, int q) {
  if (!plan->exec || plan->nbuckets - 1 >= kSideStreams) return nullptr;
  (void)q;
  return static_cast<Exec*>(plan->exec)->side[kSideStreams - 1];
}
static hipError_t fork_streams(const vecchia_plan* plan, hipStream_t s) {
  Exec* ex = static_cast<Exec*>(plan->exec);
  hipError_t e = hipEventRecord(ex->fork, s);
  for (int k = 0; k < kSideStreams && e == hipSuccess; ++k) e = hipStreamWaitEvent(ex->side[k], ex->fork, 0);
  return e;
}
static hipError_t join_streams(const vecchia_plan* plan, hipStream_t s) {
  Exec* ex = static_cast<Exec*>(plan->exec);
  hipError_t e = hipSuccess;
  for (int k = 0; k < kSideStreams && e == hipSuccess; ++k) {
    e = hipEventRecord(ex->join[k], ex->side[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ex->join[k], 0);
  }
  return e;
}

// -------------------------------------------------------------- timing ----

namespace {
struct TimingRec {
  int bucket;
  hipEvent_t e0, e1;
};
struct Timing {
  std::vector<TimingRec> recs;
};
inline hipError_t time_begin(const vecchia_plan* plan, int q, hipStream_t s, TimingRec& r) {
  r.bucket = q;
  r.e0 = r.e1 = nullptr;
  if (!plan->timing) return hipSuccess;
  hipError_t e = hipEventCreate(&r.e0);
  if (e == hipSuccess) e = hipEventCreate(&r.e1);
  if (e == hipSuccess) e = hipEventRecord(r.e0, s);
  return e;
}
inline hipError_t time_end(const vecchia_plan* plan, hipStream_t s, TimingRec& r) {
  if (!plan->timing) return hipSuccess;
  hipError_t e = hipEventRecord(r.e1, s);
  static_cast<Timing*>(plan->timing)->recs.push_back(r);
  return e;
}
void timing_clear(Timing* t) {
  for (auto& r : t->recs) {
    hipEventDestroy(r.e0);
    hipEventDestroy(r.e1);
  }
  t->recs.clear();
}
}  // namespace

extern "C" int vecchia_plan_destroy(vecchia_plan* plan) {
  if (!plan) return VECCHIA_EINVAL;
  vecchia_plan_set_timing(plan, 0);
  if (plan->exec) {
    Exec* ex = static_cast<Exec*>(plan->exec);
    for (int k = 0; k < kSideStreams; ++k) {
      if (ex->side[k]) {
        hipStreamSynchronize(ex->side[k]);
        hipStreamDestroy(ex->side[k]);
      }
      if (ex->join[k]) hipEventDestroy(ex->join[k]);
    }
    if (ex->fork) hipEventDestroy(ex->fork);
    if (ex->mark) hipEventDestroy(ex->mark);
    delete ex;
    plan->exec = nullptr;
  }
  return VECCHIA_OK;
}

extern "C" int vecchia_plan_set_timing(vecchia_plan* plan, int enable) {
  if (!plan) return VECCHIA_EINVAL;
  if (enable && !plan->timing) plan->timing = new Timing();
  if (!enable && plan->timing) {
    timing_clear(static_cast<Timing*>(plan->timing));
    delete static_cast<Timing*>(plan->timing);
    plan->timing = nullptr;
  }
  return VECCHIA_OK;
}

extern "C" int vecchia_plan_timing(vecchia_plan* plan, double* ms, int64_t* launches, int reset) {
  if (!plan || !ms || !launches) return VECCHIA_EINVAL;
  for (int q = 0; q <= plan->nbuckets; ++q) {
    ms[q] = 0.0;
    launches[q] = 0;
  }
  if (!plan->timing) return VECCHIA_OK;
  Timing* t = static_cast<Timing*>(plan->timing);
  for (auto& r : t->recs) {
    VCHECK_HIP(hipEventSynchronize(r.e1));
    float f = 0.f;
    VCHECK_HIP(hipEventElapsedTime(&f, r.e0, r.e1));
    ms[r.bucket] += (double)f;
    launches[r.bucket] += 1;
  }
  if (reset) timing_clear(t);
  return VECCHIA_OK;
}

// Bytes of the large-block slots at the start of the auxiliary workspace (the
// one-wave adjoint's tile buffer follows them).
static size_t large_bytes(const vecchia_plan* plan) {
  return plan->nlarge > 0 ? (size_t)plan->large_slots * (size_t)plan->large_slot_elems * sizeof(double) : 0;
}

// Smallest auxiliary workspace a plan can run with: every large-block slot,
// and one work item's FP64 factor tiles of the largest one-wave class (the
// adjoint then runs one item per launch).
static size_t aux_min_bytes(const vecchia_plan* plan) {
  size_t item = 0;
  if (plan->engine == kEngineMfma && plan->kind == 0)
    for (int q = 0; q < plan->nbuckets; ++q) {
      const int g = plan->bucket_cfg[q] + 1;
      if (plan->bucket_cfg[q] != kLargeCfg && wave_fits(g, false) && !wave_regadj(g, false, plan->bucket_lmax[q]) &&
          wave_tile_bytes(g, false) > item)
        item = wave_tile_bytes(g, false);
    }
  return large_bytes(plan) + item;
}

extern "C" int vecchia_plan_attach_aux(vecchia_plan* plan, void* aux_workspace, size_t bytes) {
  if (!plan) return VECCHIA_EINVAL;
  if (plan->aux_ws_bytes == 0) return VECCHIA_OK;
  if (!aux_workspace) return VECCHIA_EINVAL;
  if (bytes < aux_min_bytes(plan)) return VECCHIA_ENOMEM;
  plan->aux_ws = aux_workspace;
  // a smaller buffer than the plan asked for runs the adjoint in more launches
  if (bytes < plan->aux_ws_bytes) plan->aux_ws_bytes = bytes;
  return VECCHIA_OK;
}

static LargeArgs as_large(const FwdArgs& f, const vecchia_plan* plan) {
  LargeArgs a;
  memset(&a, 0, sizeof(a));
  a.locs = f.locs;
  a.y = f.y;
  a.block_ptr = f.block_ptr;
  a.nbr_ptr = f.nbr_ptr;
  a.nbr_idx = f.nbr_idx;
  a.sched = f.sched;
  a.list = f.list;
  a.list_count = f.list_count;
  a.nsched = f.nsched;
  a.ntheta = f.ntheta;
  a.bc = f.bc;
  a.d = f.d;
  a.fp32_guard = f.fp32_guard;
  a.flag_or = f.flag_or;
  a.ws = plan->aux_ws;
  a.slot_elems = plan->large_slot_elems;
  a.partial = f.partial;
  a.flag = f.flag;
  a.gpart = nullptr;
  return a;
}

// Large-block arguments of a gradient launch.
static LargeArgs as_large(const AdjArgs& f, const vecchia_plan* plan) {
  FwdArgs w;
  memset(&w, 0, sizeof(w));
  w.locs = f.locs;
  w.y = f.y;
  w.block_ptr = f.block_ptr;
  w.nbr_ptr = f.nbr_ptr;
  w.nbr_idx = f.nbr_idx;
  w.sched = f.sched;
  w.list = f.list;
  w.list_count = f.list_count;
  w.nsched = f.nsched;
  w.ntheta = f.ntheta;
  w.bc = f.bc;
  w.d = f.d;
  w.fp32_guard = f.fp32_guard;
  w.flag_or = f.flag_or;
  w.partial = f.partial;
  w.flag = f.flag;
  LargeArgs a = as_large(w, plan);
  a.gpart = f.gpart;
  return a;
}

// -------------------------------------------------------------- loglik ----

static int check_common(const vecchia_plan* plan, const double* locs, const double* y, int32_t d,
                        const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                        const vecchia_theta* theta, int32_t ntheta, int32_t precision) {
  if (!plan || !plan->ws || !locs || !y || !block_ptr || !nbr_ptr || !nbr_idx || !theta) return VECCHIA_EINVAL;
  if (plan->kind != 0) return VECCHIA_EINVAL;   // a prediction plan
  if (d < 1 || d > 3 || ntheta < 1 || ntheta > plan->max_theta) return VECCHIA_EINVAL;
  if (precision != VECCHIA_FP64 && precision != VECCHIA_FP32_BULK && precision != VECCHIA_FP32_BULK_FORCE_REFACTOR)
    return VECCHIA_EINVAL;
  for (int t = 0; t < ntheta; ++t) {
    ThetaDev td;
    const int st = theta_status(theta[t], d, td);
    if (st) return st;
    // the Bessel form is evaluated by the one-wave kernels only
    if (td.nu_code == 3 && (plan->engine != kEngineMfma || plan->nlarge > 0)) return VECCHIA_EUNSUPPORTED;
  }
  return VECCHIA_OK;
}

int bv::check_loglik_args(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                          const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                          const vecchia_theta* theta, int32_t ntheta, int32_t precision, const double* loglik,
                          bool need_aux) {
  int st = check_common(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, theta, ntheta, precision);
  if (st) return st;
  if (!loglik) return VECCHIA_EINVAL;
  if (need_aux && plan->aux_ws_bytes > 0 && !plan->aux_ws) return VECCHIA_ENOMEM;
  return VECCHIA_OK;
}

// The value path of vecchia_loglik with its per-call buffers (per-block terms,
// flags, compaction lists and counts) passed in; arguments already checked.
int bv::loglik_run(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                   const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                   const vecchia_theta* theta, int32_t ntheta, int32_t precision, double* loglik,
                   int32_t* counters, double* partial, const CallBuffers& cb, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int bc = (int)plan->bc;
  const bool fp32 = precision != VECCHIA_FP64;
  const int* sched = at<int>(plan->ws, plan->off_sched);
  double* part = cb.partial;
  int* flag = cb.flag;
  int* list = cb.list;
  int* count = cb.count;

  for (int t0 = 0; t0 < ntheta; t0 += kMaxThetaPerLaunch) {
    const int nt = ntheta - t0 < kMaxThetaPerLaunch ? ntheta - t0 : kMaxThetaPerLaunch;
    ThetaPack thp;
    memset(&thp, 0, sizeof(thp));
    for (int t = 0; t < nt; ++t) theta_to_dev(theta[t0 + t], d, thp.t[t]);
    FwdArgs a;
    memset(&a, 0, sizeof(a));
    a.locs = locs_perm;
    a.y = y_perm;
    a.block_ptr = block_ptr;
    a.nbr_ptr = nbr_ptr;
    a.nbr_idx = nbr_idx;
    a.ntheta = nt;
    a.bc = bc;
    a.d = d;
    a.fp32_guard = precision == VECCHIA_FP32_BULK_FORCE_REFACTOR ? 2 : (fp32 ? 1 : 0);
    a.partial = part;
    a.flag = flag;
    const bool conc = plan->exec != nullptr;   // size classes run concurrently
    TimingRec span;
    VCHECK_HIP(time_begin(plan, plan->nbuckets, s, span));
    if (conc) VCHECK_HIP(fork_streams(plan, s));
    // largest blocks first: their long single-wave items start early and the
    // smaller classes fill in around them
    for (int q = plan->nbuckets - 1; q >= 0; --q) {
      const int ns = (int)(plan->bucket_off[q + 1] - plan->bucket_off[q]);
      const hipStream_t sq = class_stream(plan, q, s, conc);
      a.sched = sched + plan->bucket_off[q];
      a.nsched = ns;
      TimingRec tr;
      VCHECK_HIP(time_begin(plan, q, sq, tr));
      if (plan->bucket_cfg[q] == kLargeCfg) {
        const int g = ns * nt < plan->large_slots ? ns * nt : plan->large_slots;
        VCHECK_HIP(launch_large(fp32, false, as_large(a, plan), thp, g, sq));
      } else {
        if (plan->engine == kEngineTiles)
          VCHECK_HIP(launch_forward(plan->bucket_cfg[q], fp32, a, thp, ns * nt, sq));
        else
          VCHECK_ST(launch_mfma_class(plan, q, fp32, 0, as_adj(a, plan), thp, ns * nt, sq, nullptr, 0));
      }
      VCHECK_HIP(time_end(plan, sq, tr));
    }
    if (conc) VCHECK_HIP(join_streams(plan, s));
    VCHECK_HIP(time_end(plan, s, span));
    if (fp32) {
      // FP32 guard: compact flagged (theta, block) pairs per size class, re-run them in FP64
      VCHECK_HIP(launch_fill_int(count, plan->nbuckets, 0, s));
      for (int q = 0; q < plan->nbuckets; ++q) {
        const int ns = (int)(plan->bucket_off[q + 1] - plan->bucket_off[q]);
        VCHECK_HIP(launch_compact_flagged(sched + plan->bucket_off[q], ns, nt, bc, flag,
                                          list + plan->bucket_off[q] * nt, count + q, s));
      }
      FwdArgs r = a;
      r.fp32_guard = 0;
      r.flag_or = 5;   // re-run in FP64 (4); the guard bit (1) that listed it stays set
      for (int q = 0; q < plan->nbuckets; ++q) {
        const int ns = (int)(plan->bucket_off[q + 1] - plan->bucket_off[q]);
        r.list = list + plan->bucket_off[q] * nt;
        r.list_count = count + q;
        const int cap = ns * nt;
        if (plan->bucket_cfg[q] == kLargeCfg)
          VCHECK_HIP(launch_large(false, false, as_large(r, plan), thp, cap < plan->large_slots ? cap : plan->large_slots,
                                  s));
        else if (plan->engine == kEngineTiles)
          VCHECK_HIP(launch_forward(plan->bucket_cfg[q], false, r, thp, cap < 256 ? cap : 256, s));
        else
          VCHECK_ST(launch_mfma_class(plan, q, false, 0, as_adj(r, plan), thp, cap, s, nullptr, 0));
      }
    }
    VCHECK_HIP(launch_reduce_partials(part, flag, bc, nt, fp32 ? 0 : 1, loglik + t0,
                                      counters ? counters + 2 * t0 : nullptr, s));
    if (partial)
      VCHECK_HIP(hipMemcpyAsync(partial + (size_t)t0 * bc, part, sizeof(double) * (size_t)nt * bc,
                                hipMemcpyDeviceToDevice, s));
  }
  return VECCHIA_OK;
}

extern "C" int vecchia_loglik(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                              const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                              const vecchia_theta* theta, int32_t ntheta, int32_t precision, double* loglik,
                              int32_t* counters, double* partial, void* stream) {
  const int st = check_loglik_args(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, theta, ntheta, precision,
                                   loglik, true);
  if (st) return st;
  CallBuffers cb;
  cb.partial = at<double>(plan->ws, plan->off_partial);
  cb.flag = at<int>(plan->ws, plan->off_flag);
  cb.list = at<int>(plan->ws, plan->off_list);
  cb.count = at<int>(plan->ws, plan->off_count);
  return loglik_run(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, theta, ntheta, precision, loglik,
                    counters, partial, cb, stream);
}

// ----------------------------------------------------------- loglik_grad --

// Value and gradient; with dnu (and optionally gpartial_nu) the derivative in
// nu as well, through the Bessel-form kernels.
static int loglik_grad_run(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                           const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                           const vecchia_theta* theta, int32_t ntheta, int32_t precision, double* loglik,
                           double* grad, double* dnu, int32_t* counters, double* partial, double* gpartial,
                           double* gpartial_nu, void* stream) {
  int st = check_common(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, theta, ntheta, precision);
  if (st) return st;
  if (!loglik || !grad) return VECCHIA_EINVAL;
  // d / d nu: the Bessel form runs on the one-wave kernels only
  if (dnu && (plan->engine != kEngineMfma || plan->nlarge > 0)) return VECCHIA_EUNSUPPORTED;
  // The adjoint of blocks above the one-wave limit (bv_large_kernel<T, true>)
  // is switched off: its first GPU run ended with a device fault whose cause
  // has not been found (a CPU emulation of its indexing stays in bounds).
  if (plan->nlarge > 0) return VECCHIA_EUNSUPPORTED;
  if (plan->aux_ws_bytes > 0 && !plan->aux_ws) return VECCHIA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  const int bc = (int)plan->bc;
  void* ws = plan->ws;
  const bool fp32 = precision != VECCHIA_FP64;
  const int* sched = at<int>(ws, plan->off_sched);
  double* part = at<double>(ws, plan->off_partial);
  double* gpart = at<double>(ws, plan->off_grad);
  double* gnu = dnu ? gpart + (size_t)bc * plan->max_theta * 3 : nullptr;
  const size_t lbytes = large_bytes(plan);
  char* tile_ws = static_cast<char*>(plan->aux_ws) + lbytes;   // after the large-block slots
  const size_t tile_ws_bytes = plan->aux_ws_bytes - lbytes;
  int* flag = at<int>(ws, plan->off_flag);
  int* list = at<int>(ws, plan->off_list);
  int* count = at<int>(ws, plan->off_count);

  for (int t0 = 0; t0 < ntheta; t0 += kMaxThetaPerLaunch) {
    const int nt = ntheta - t0 < kMaxThetaPerLaunch ? ntheta - t0 : kMaxThetaPerLaunch;
    ThetaPack thp;
    memset(&thp, 0, sizeof(thp));
    for (int t = 0; t < nt; ++t) theta_to_dev(theta[t0 + t], d, thp.t[t]);
    AdjArgs a;
    memset(&a, 0, sizeof(a));
    a.locs = locs_perm;
    a.y = y_perm;
    a.block_ptr = block_ptr;
    a.nbr_ptr = nbr_ptr;
    a.nbr_idx = nbr_idx;
    a.ntheta = nt;
    a.bc = bc;
    a.d = d;
    a.fp32_guard = precision == VECCHIA_FP32_BULK_FORCE_REFACTOR ? 2 : (fp32 ? 1 : 0);
    a.ldx = 0;   // set per size class
    a.partial = part;
    a.gpart = gpart;
    a.gnu = gnu;
    a.flag = flag;
    // the one-wave adjoint's tile buffer is split among the size classes so
    // that they can run concurrently; if it is too small they run in turn
    size_t off[VECCHIA_MAX_BUCKETS + 1] = {0};
    for (int q = 0; q < plan->nbuckets; ++q) {
      const int g = plan->bucket_cfg[q] + 1;
      const size_t ns = (size_t)(plan->bucket_off[q + 1] - plan->bucket_off[q]);
      const bool tiles = plan->engine == kEngineMfma && plan->bucket_cfg[q] != kLargeCfg && wave_fits(g, fp32) &&
                         !wave_regadj(g, fp32, plan->bucket_lmax[q]);
      off[q + 1] = off[q] + (tiles ? ns * nt * wave_tile_bytes(g, fp32) : 0);
    }
    const bool conc = plan->exec != nullptr && off[plan->nbuckets] <= tile_ws_bytes;
    // the largest class waits for the first factorisation launch of the split
    // (two-launch) class with the most blocks, so that the long one-wave-per-SIMD
    // factorisation items start first and the fine-grained class fills in last
    int qmark = -1;
    if (conc && plan->engine == kEngineMfma && kMarkSplit)
      for (int q = 0; q < plan->nbuckets; ++q)
        if (q != plan->bucket_main && plan->bucket_cfg[q] != kLargeCfg && class_wave_mode(plan, q, fp32, true) == 23 &&
            (qmark < 0 || plan->bucket_off[q + 1] - plan->bucket_off[q] >
                              plan->bucket_off[qmark + 1] - plan->bucket_off[qmark]))
          qmark = q;
    TimingRec span;
    VCHECK_HIP(time_begin(plan, plan->nbuckets, s, span));
    if (conc) VCHECK_HIP(fork_streams(plan, s));
    // largest blocks first: their long single-wave items start early and the
    // smaller classes fill in around them
    for (int q = plan->nbuckets - 1; q >= 0; --q) {
      const int ns = (int)(plan->bucket_off[q + 1] - plan->bucket_off[q]);
      const hipStream_t sq = class_stream(plan, q, s, conc);
      a.sched = sched + plan->bucket_off[q];
      a.nsched = ns;
      TimingRec tr;
      VCHECK_HIP(time_begin(plan, q, sq, tr));
      if (plan->bucket_cfg[q] == kLargeCfg) {
        const int g = ns * nt < plan->large_slots ? ns * nt : plan->large_slots;
        VCHECK_HIP(launch_large(fp32, true, as_large(a, plan), thp, g, sq));
      } else if (plan->engine == kEngineTiles) {
        VCHECK_ST(launch_tiles_adjoint(plan, q, fp32, a, thp, ns * nt, sq));
      } else if (conc) {
        Exec* ex = static_cast<Exec*>(plan->exec);
        if (q == plan->bucket_main && qmark >= 0) VCHECK_HIP(hipStreamWaitEvent(sq, ex->mark, 0));
        VCHECK_ST(launch_mfma_class(plan, q, fp32, 1, a, thp, ns * nt, sq, tile_ws + off[q], off[q + 1] - off[q],
                                    spare_stream(plan, q), q == qmark ? ex->mark : nullptr));
      } else {
        VCHECK_ST(launch_mfma_class(plan, q, fp32, 1, a, thp, ns * nt, sq, tile_ws, tile_ws_bytes));
      }
      VCHECK_HIP(time_end(plan, sq, tr));
    }
    if (conc) VCHECK_HIP(join_streams(plan, s));
    VCHECK_HIP(time_end(plan, s, span));
    if (fp32) {
      VCHECK_HIP(launch_fill_int(count, plan->nbuckets, 0, s));
      for (int q = 0; q < plan->nbuckets; ++q) {
        const int ns = (int)(plan->bucket_off[q + 1] - plan->bucket_off[q]);
        VCHECK_HIP(launch_compact_flagged(sched + plan->bucket_off[q], ns, nt, bc, flag,
                                          list + plan->bucket_off[q] * nt, count + q, s));
      }
      AdjArgs r = a;
      r.fp32_guard = 0;
      r.flag_or = 5;   // re-run in FP64 (4); the guard bit (1) that listed it stays set
      for (int q = 0; q < plan->nbuckets; ++q) {
        const int ns = (int)(plan->bucket_off[q + 1] - plan->bucket_off[q]);
        r.list = list + plan->bucket_off[q] * nt;
        r.list_count = count + q;
        const int cap = ns * nt;
        if (plan->bucket_cfg[q] == kLargeCfg)
          VCHECK_HIP(launch_large(false, true, as_large(r, plan), thp, cap < plan->large_slots ? cap : plan->large_slots,
                                  s));
        else if (plan->engine == kEngineTiles)
          VCHECK_ST(launch_tiles_adjoint(plan, q, false, r, thp, cap < 256 ? cap : 256, s));
        else
          VCHECK_ST(launch_mfma_class(plan, q, false, 1, r, thp, cap, s, tile_ws, tile_ws_bytes));
      }
    }
    VCHECK_HIP(launch_reduce_partials(part, flag, bc, nt, fp32 ? 0 : 1, loglik + t0,
                                      counters ? counters + 2 * t0 : nullptr, s));
    VCHECK_HIP(launch_reduce_vec(gpart, bc, 3, nt, grad + 3 * t0, s));
    if (gnu) VCHECK_HIP(launch_reduce_vec(gnu, bc, 1, nt, dnu + t0, s));
    if (partial)
      VCHECK_HIP(hipMemcpyAsync(partial + (size_t)t0 * bc, part, sizeof(double) * (size_t)nt * bc,
                                hipMemcpyDeviceToDevice, s));
    if (gpartial)
      VCHECK_HIP(hipMemcpyAsync(gpartial + (size_t)t0 * bc * 3, gpart, sizeof(double) * (size_t)nt * bc * 3,
                                hipMemcpyDeviceToDevice, s));
    if (gnu && gpartial_nu)
      VCHECK_HIP(hipMemcpyAsync(gpartial_nu + (size_t)t0 * bc, gnu, sizeof(double) * (size_t)nt * bc,
                                hipMemcpyDeviceToDevice, s));
  }
  return VECCHIA_OK;
}

extern "C" int vecchia_loglik_grad(const vecchia_plan* plan, const double* locs_perm, const double* y_perm,
                                   int32_t d, const int32_t* block_ptr, const int32_t* nbr_ptr,
                                   const int32_t* nbr_idx, const vecchia_theta* theta, int32_t ntheta,
                                   int32_t precision, double* loglik, double* grad, int32_t* counters,
                                   double* partial, double* gpartial, void* stream) {
  return loglik_grad_run(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, theta, ntheta, precision, loglik,
                         grad, nullptr, counters, partial, gpartial, nullptr, stream);
}

extern "C" int vecchia_loglik_grad_nu(const vecchia_plan* plan, const double* locs_perm, const double* y_perm,
                                      int32_t d, const int32_t* block_ptr, const int32_t* nbr_ptr,
                                      const int32_t* nbr_idx, const vecchia_theta* theta, int32_t ntheta,
                                      int32_t precision, double* loglik, double* grad, double* dnu,
                                      int32_t* counters, double* partial, double* gpartial, double* gpartial_nu,
                                      void* stream) {
  if (!dnu) return VECCHIA_EINVAL;
  return loglik_grad_run(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, theta, ntheta, precision, loglik,
                         grad, dnu, counters, partial, gpartial, gpartial_nu, stream);
}

// ------------------------------------------------------------- predict ----

extern "C" int vecchia_predict(const vecchia_plan* plan, const double* locs_obs, const double* y_obs,
                               const double* locs_new, int32_t d, const int32_t* block_ptr, const int32_t* nbr_ptr,
                               const int32_t* nbr_idx, const vecchia_theta* theta, double* mean, double* var,
                               double* cov, int32_t ldc, void* stream) {
  if (!plan || plan->kind != 1 || !plan->ws || !locs_obs || !y_obs || !locs_new || !block_ptr || !nbr_ptr ||
      !nbr_idx || !theta || !mean || !var)
    return VECCHIA_EINVAL;
  if (d < 1 || d > 3 || (cov && ldc < plan->lmax)) return VECCHIA_EINVAL;
  ThetaPack thp;
  memset(&thp, 0, sizeof(thp));
  const int st = theta_status(*theta, d, thp.t[0]);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  AdjArgs a;
  memset(&a, 0, sizeof(a));
  a.locs = locs_obs;
  a.y = y_obs;
  a.block_ptr = block_ptr;
  a.nbr_ptr = nbr_ptr;
  a.nbr_idx = nbr_idx;
  a.ntheta = 1;
  a.bc = (int)plan->bc;
  a.d = d;
  a.locs2 = locs_new;
  a.out_mean = mean;
  a.out_var = var;
  a.out_cov = cov;
  a.ldc = cov ? ldc : 0;
  a.gen = thp.t[0].nu_code == 3;
  const int* sched = at<int>(plan->ws, plan->off_sched);
  const bool conc = plan->exec != nullptr;
  TimingRec span;
  VCHECK_HIP(time_begin(plan, plan->nbuckets, s, span));
  if (conc) VCHECK_HIP(fork_streams(plan, s));
  for (int q = plan->nbuckets - 1; q >= 0; --q) {
    const int ns = (int)(plan->bucket_off[q + 1] - plan->bucket_off[q]);
    const hipStream_t sq = class_stream(plan, q, s, conc);
    a.sched = sched + plan->bucket_off[q];
    a.nsched = ns;
    TimingRec tr;
    VCHECK_HIP(time_begin(plan, q, sq, tr));
    VCHECK_HIP(launch_wave(plan->bucket_cfg[q] + 1, false, 4, a, thp, ns, sq));
    VCHECK_HIP(time_end(plan, sq, tr));
  }
  if (conc) VCHECK_HIP(join_streams(plan, s));
  VCHECK_HIP(time_end(plan, s, span));
  return VECCHIA_OK;
}

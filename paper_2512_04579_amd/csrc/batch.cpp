// Batched GN-MPPI (Alg. 1) over many independent chain MPC instances of
// uneven size: the host-side plan (workspace layout, per-instance
// descriptors, work lists per step and shape class) and the C ABI that
// prepares it and enqueues one iteration.
//
// The plan is a pure function of (shared problem, instances, settings,
// tuning), so gnmppi_batch_iteration recomputes it on the host instead of
// keeping state: the library stays stateless and an iteration can be
// captured into a HIP graph (it only enqueues kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "batch.hpp"
#include "gnmppi.h"
#include "launch.hpp"

namespace gnm {
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
inline int cdiv(int a, int b) { return (a + b - 1) / b; }

constexpr int kCus = 256;  // MI355X compute units: the persistent grids are sized per CU

// Steps of one iteration in launch order; each is split by its shape class.
enum Step {
  kSample, kGramW, kReduceG, kRollout, kNominal, kFused, kSplit, kContractS, kReduceS, kSweepG,
  kGramH, kReduceH, kSweepH, kLine, kSteps
};

// Rollout modes (gnmppi_batch_tuning.rollout_mode): residuals through HBM
// (lane-group rollout, then the BF16x3 contraction) or the fused kernel
// (one lane per sample, contraction on the MFMA, no residuals in HBM).
constexpr int kModeDefault = 0, kModeUnfused = 1, kModeFused = 2;

struct PlanLaunch {
  Step step;
  int cls;       // template parameter of the class (G, NT or R); 0 if none
  size_t first;  // index of the first item
  int count, blocks;
};

struct Plan {
  std::vector<BatchInst> inst;  // host copy, device pointers filled in
  std::vector<BatchItem> items;
  std::vector<PlanLaunch> launches;
  size_t inst_off = 0, items_off = 0, alpha_off = 0, total = 0;
  int N_max = 0;
};

bool instance_ok(const gnmppi_batch_instance& b) {
  if (b.n_masses < 3 || b.n_masses > 16 || b.N < 1 || b.N > 80) return false;
  if (b.K < 2 || (b.K % 2) != 0 || b.K / 2 < 2 * b.N || b.K > (1 << 16)) return false;
  return b.x0 && b.q && b.r && b.x_ref && b.U && b.status && b.info;
}

bool settings_ok(const gnmppi_batch_settings* s) {
  return s && s->n_alpha >= 1 && s->n_alpha <= 64 && s->gamma > 0.0 && s->gamma < 1.0 &&
         s->lm_lambda >= 0.0 && std::isfinite(s->lm_lambda);
}

gnmppi_batch_tuning effective(const gnmppi_batch_tuning* t) {
  // defaults: the autotuner's pick for 1024 uneven chain instances
  gnmppi_batch_tuning d{64, 16, 1, 32, kModeFused};
  if (t) {
    if (t->rollout_mode == kModeUnfused || t->rollout_mode == kModeFused)
      d.rollout_mode = t->rollout_mode;
    if (t->rollout_blocks_per_cu > 0) d.rollout_blocks_per_cu = t->rollout_blocks_per_cu;
    if (t->contract_blocks_per_cu > 0) d.contract_blocks_per_cu = t->contract_blocks_per_cu;
    if (t->contract_ksplit > 0) d.contract_ksplit = t->contract_ksplit;
    if (t->small_blocks_per_cu > 0) d.small_blocks_per_cu = t->small_blocks_per_cu;
  }
  return d;
}

// Builds the plan; `base` is the device address of the workspace (null for a
// size query).
Plan make_plan(int count, const gnmppi_batch_instance* in, const gnmppi_batch_settings* set,
               const gnmppi_batch_tuning* tune_in, char* base) {
  const gnmppi_batch_tuning tune = effective(tune_in);
  Plan pl;
  pl.inst.resize(count);
  size_t off = 0;
  pl.inst_off = off;
  off = align_up(off + sizeof(BatchInst) * count);
  // items are counted first so that their region can precede the buffers
  std::vector<int> tiles[kSteps];
  for (auto& t : tiles) t.resize(count);
  for (int i = 0; i < count; ++i) {
    const gnmppi_batch_instance& b = in[i];
    BatchInst& d = pl.inst[i];
    d.M = b.n_masses;
    d.N = b.N;
    d.K = b.K;
    d.n = 2 * b.N;
    d.m = b.N * (4 * b.n_masses + 2);
    d.npad = cdiv(d.n, 16) * 16;
    d.kpad = cdiv(d.K, 32) * 32;
    const bool fused = tune.rollout_mode == kModeFused;
    const int ksteps = cdiv(d.K, 32);
    if (fused) {
      // one partial sum of S per block of kFusedPairs antithetic pairs
      d.nsplit = cdiv(d.K / 2, kFusedPairs);
      d.split_len = 2 * kFusedPairs;
    } else {
      const int ns = std::max(1, std::min(tune.contract_ksplit, ksteps));
      const int spl = cdiv(ksteps, ns);
      d.nsplit = cdiv(ksteps, spl);
      d.split_len = spl * 32;
    }
    d.gsplit = 1;
    // the fused kernel forms G = W W^T with S: n more rows per k-slice
    d.grows = fused ? d.n : 0;
    d.gsplit_len = ksteps * 32;
    d.hsplit = std::max(1, std::min(16, cdiv(d.m, 128)));
    d.hchunk = cdiv(cdiv(d.m, d.hsplit), 4) * 4;
    d.hsplit = cdiv(d.m, d.hchunk);
    d.ldw = d.ldr = cdiv(d.K, 64) * 64;
    d.seed = set->seed + static_cast<uint64_t>(i);
    pl.N_max = std::max(pl.N_max, d.N);
    tiles[kSample][i] = batch_sample_tiles(d.n, d.K);
    tiles[kGramW][i] = fused ? 0 : batch_contract_row_blocks(d.n) * d.gsplit;
    tiles[kReduceG][i] = fused ? 0 : d.n;
    tiles[kSweepG][i] = 1;
    tiles[kRollout][i] = fused ? 0 : batch_rollout_tiles(d.M, d.K);
    tiles[kNominal][i] = fused ? 1 : 0;
    tiles[kFused][i] = fused ? d.nsplit : 0;
    tiles[kSplit][i] = 0;  // the sampler writes the bf16 planes itself
    tiles[kContractS][i] = fused ? 0 : batch_bf16_row_blocks(d.m) * d.nsplit;
    // one k-slice: the partial sum already is S (no reduction)
    // (with G rows the reduction also writes G in FP64, so it always runs)
    tiles[kReduceS][i] =
        d.nsplit > 1 || d.grows > 0 ? cdiv(d.m + d.grows, 16) * cdiv(d.npad, 64) : 0;
    tiles[kGramH][i] = d.hsplit;
    tiles[kReduceH][i] = d.n + 1;
    tiles[kSweepH][i] = 1;
    tiles[kLine][i] = 1;
  }
  // instances in decreasing order of work, so that persistent blocks pick up
  // the long items first
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double wa = static_cast<double>(pl.inst[a].m) * pl.inst[a].K;
    const double wb = static_cast<double>(pl.inst[b].m) * pl.inst[b].K;
    return wa > wb;
  });
  auto cls_of = [&](Step s, const BatchInst& d) -> int {
    switch (s) {
      case kGramW: case kContractS: return cdiv(d.n, 16);
      case kSweepG: return cdiv(d.n, 16);
      case kGramH: case kSweepH: return cdiv(d.n + 1, 16);
      case kRollout: case kNominal: case kLine: return batch_chain_group(d.M);
      case kFused: return 0;  // one launch for every chain length
      default: return 0;
    }
  };
  auto cap = [&](Step s) -> int {
    switch (s) {
      case kRollout: return tune.rollout_blocks_per_cu * kCus;
      case kContractS: return tune.contract_blocks_per_cu * kCus;
      case kSweepG: case kSweepH: case kLine: case kNominal: return 8 * kCus;
      case kFused: return kCus;  // one 512-thread block per CU (157 KB of LDS)
      default: return tune.small_blocks_per_cu * kCus;
    }
  };
  for (int s = 0; s < kSteps; ++s) {
    std::map<int, std::vector<int>> classes;
    for (int i : order) classes[cls_of(static_cast<Step>(s), pl.inst[i])].push_back(i);
    for (auto& kv : classes) {
      PlanLaunch L{static_cast<Step>(s), kv.first, pl.items.size(), 0, 0};
      for (int i : kv.second)
        for (int t = 0; t < tiles[s][i]; ++t) pl.items.push_back(BatchItem{i, t});
      L.count = static_cast<int>(pl.items.size() - L.first);
      if (L.count == 0) continue;
      L.blocks = std::max(1, std::min(L.count, cap(static_cast<Step>(s))));
      pl.launches.push_back(L);
    }
  }
  pl.items_off = off;
  off = align_up(off + sizeof(BatchItem) * pl.items.size());
  pl.alpha_off = off;
  off = align_up(off + sizeof(float) * 64);
  for (int i = 0; i < count; ++i) {
    BatchInst& d = pl.inst[i];
    const gnmppi_batch_instance& b = in[i];
    const int P = d.n + 1;
    auto take = [&](size_t bytes) -> char* {
      char* p = base ? base + off : nullptr;
      off = align_up(off + bytes);
      return p;
    };
    d.x0 = static_cast<const float*>(b.x0);
    d.q = static_cast<const float*>(b.q);
    d.r = static_cast<const float*>(b.r);
    d.xref = static_cast<const float*>(b.x_ref);
    d.U = static_cast<float*>(b.U);
    d.status = b.status;
    d.info = b.info;
    d.W = reinterpret_cast<float*>(take(sizeof(float) * d.n * d.ldw));
    // the fused path keeps the residuals on chip
    d.R = tune.rollout_mode == kModeFused
              ? nullptr
              : reinterpret_cast<float*>(take(sizeof(float) * static_cast<size_t>(d.m) * d.ldr));
    d.C = nullptr;  // the GN-MPPI step never reads the perturbed columns' costs
    d.r0 = reinterpret_cast<float*>(take(sizeof(float) * d.m));
    d.c0 = reinterpret_cast<float*>(take(sizeof(float)));
    d.dU = reinterpret_cast<float*>(take(sizeof(float) * d.n));
    d.part = reinterpret_cast<float*>(
        take(sizeof(float) * static_cast<size_t>(d.nsplit) * (d.m + d.grows) * d.npad));
    d.S = d.nsplit > 1 || d.grows > 0
              ? reinterpret_cast<float*>(take(sizeof(float) * static_cast<size_t>(d.m) * d.npad))
              : d.part;
    d.gpart = d.grows > 0 ? nullptr
                          : reinterpret_cast<float*>(take(sizeof(float) *
                                                          static_cast<size_t>(d.gsplit) * d.n *
                                                          d.npad));
    d.Ginv = reinterpret_cast<float*>(take(sizeof(float) * d.n * d.npad));
    d.Wh = reinterpret_cast<__bf16*>(take(2 * static_cast<size_t>(d.n) * d.kpad));
    d.Wl = reinterpret_cast<__bf16*>(take(2 * static_cast<size_t>(d.n) * d.kpad));
    d.Gsum = reinterpret_cast<double*>(take(sizeof(double) * d.n * d.n));
    d.hpart = reinterpret_cast<double*>(take(sizeof(double) * static_cast<size_t>(d.hsplit) * P * P));
    d.Hsum = reinterpret_cast<double*>(take(sizeof(double) * P * P));
    d.alpha = base ? reinterpret_cast<float*>(base + pl.alpha_off) : nullptr;
  }
  pl.total = off;
  return pl;
}

int validate(const gnmppi_problem* shared, int32_t count, const gnmppi_batch_instance* inst,
             const gnmppi_batch_settings* set) {
  if (shared == nullptr || shared->model != GNMPPI_MODEL_CHAIN || shared->dtype != GNMPPI_F32)
    return GNMPPI_EINVAL;
  if (!(shared->dt > 0.0) || !(shared->mass > 0.0) || !std::isfinite(shared->k_lin) ||
      !std::isfinite(shared->k_cub))
    return GNMPPI_EINVAL;
  if (count < 1 || count > (1 << 20) || inst == nullptr || !settings_ok(set)) return GNMPPI_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!instance_ok(inst[i])) return GNMPPI_EINVAL;
  return GNMPPI_OK;
}

hipError_t run_iteration(const Plan& pl, const gnmppi_problem& shared, char* base, int it,
                         double sigma, const gnmppi_batch_settings& set, hipStream_t st) {
  const BatchInst* inst = reinterpret_cast<const BatchInst*>(base + pl.inst_off);
  const BatchItem* items = reinterpret_cast<const BatchItem*>(base + pl.items_off);
  for (const PlanLaunch& L : pl.launches) {
    const BatchLaunch bl{items + L.first, L.count, L.blocks};
    hipError_t e = hipSuccess;
    switch (L.step) {
      case kSample: e = launch_batch_sample(inst, bl, sigma, static_cast<uint64_t>(it), st); break;
      case kGramW: e = launch_batch_contract(L.cls, inst, bl, st); break;
      case kReduceG: e = launch_batch_reduce_sym(0, inst, bl, 0.0, st); break;
      case kSweepG: e = launch_batch_sweep(0, L.cls, inst, bl, st); break;
      case kRollout: e = launch_batch_rollout(L.cls, inst, bl, shared, pl.N_max, st); break;
      case kNominal: e = launch_batch_nominal(L.cls, inst, bl, shared, pl.N_max, st); break;
      case kFused: e = launch_batch_fused(inst, bl, shared, st); break;
      case kSplit: e = launch_batch_split_bf16(inst, bl, st); break;
      case kContractS: e = launch_batch_contract_bf16(L.cls, inst, bl, st); break;
      case kReduceS: e = launch_batch_reduce_rows(inst, bl, st); break;
      case kGramH: e = launch_batch_gram(L.cls, inst, bl, st); break;
      case kReduceH: e = launch_batch_reduce_sym(1, inst, bl, set.lm_lambda, st); break;
      case kSweepH: e = launch_batch_sweep(1, L.cls, inst, bl, st); break;
      case kLine:
        e = launch_batch_line_search(L.cls, inst, bl, shared, set.n_alpha, pl.N_max, st);
        break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace
}  // namespace gnm

extern "C" {

size_t gnmppi_batch_workspace(const gnmppi_problem* shared, int32_t count,
                              const gnmppi_batch_instance* inst, const gnmppi_batch_settings* set,
                              const gnmppi_batch_tuning* tune) {
  if (gnm::validate(shared, count, inst, set) != GNMPPI_OK) return 0;
  return gnm::make_plan(count, inst, set, tune, nullptr).total;
}

int gnmppi_batch_prepare(const gnmppi_problem* shared, int32_t count,
                         const gnmppi_batch_instance* inst, const gnmppi_batch_settings* set,
                         const gnmppi_batch_tuning* tune, void* work, size_t work_bytes) {
  const int v = gnm::validate(shared, count, inst, set);
  if (v != GNMPPI_OK) return v;
  if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) != 0) return GNMPPI_EINVAL;
  char* base = static_cast<char*>(work);
  const gnm::Plan pl = gnm::make_plan(count, inst, set, tune, base);
  if (work_bytes < pl.total) return GNMPPI_ENOSPACE;
  float alpha[64];
  double a = 1.0;
  for (int j = 0; j < set->n_alpha; ++j, a *= set->gamma) alpha[j] = static_cast<float>(a);
  hipError_t e = hipMemcpy(base + pl.inst_off, pl.inst.data(), sizeof(gnm::BatchInst) * count,
                           hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + pl.items_off, pl.items.data(), sizeof(gnm::BatchItem) * pl.items.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + pl.alpha_off, alpha, sizeof(float) * set->n_alpha, hipMemcpyHostToDevice);
  return e == hipSuccess ? GNMPPI_OK : GNMPPI_EHIP;
}

int gnmppi_batch_iteration(const gnmppi_problem* shared, int32_t count,
                           const gnmppi_batch_instance* inst, const gnmppi_batch_settings* set,
                           const gnmppi_batch_tuning* tune, void* work, size_t work_bytes,
                           int32_t it, double sigma, void* stream) {
  const int v = gnm::validate(shared, count, inst, set);
  if (v != GNMPPI_OK) return v;
  if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) != 0 || it < 0 ||
      !(sigma > 0.0) || !std::isfinite(sigma))
    return GNMPPI_EINVAL;
  char* base = static_cast<char*>(work);
  const gnm::Plan pl = gnm::make_plan(count, inst, set, tune, base);
  if (work_bytes < pl.total) return GNMPPI_ENOSPACE;
  const hipError_t e =
      gnm::run_iteration(pl, *shared, base, it, sigma, *set, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GNMPPI_OK : GNMPPI_EHIP;
}

}  // extern "C"

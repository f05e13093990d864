// Host side of liblb's C ABI (include/lb.h): context lifetime, device
// buffers, argument checks, kernel dispatch on the caller's stream, and
// per-kernel event timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lb.h"
#include "lb_adjoint.h"
#include "lb_fused.h"
#include "lb_kernels.h"
#include "lb_particles.h"
#include "lb_single.h"

using namespace lbd;

namespace {

enum KernelSlot : int {
  SLOT_PSI = 0,
  SLOT_COLLIDE = 1,
  SLOT_FUSED = 2,
  SLOT_ADJ_MOMENTS = 3,
  SLOT_ADJ_LOCAL = 4,
  SLOT_ADJ_R = 5,
  SLOT_PART_FORCE = 6,
  SLOT_PART_OWNER = 7,
  SLOT_PART_REMAP = 8,
  SLOT_COUNT = 9
};
const char* const kSlotNames[SLOT_COUNT] = {"psi",     "collide_push", "fused",      "adj_moments",
                                            "adj_local", "adj_r",     "part_force", "part_owner",
                                            "part_remap"};
constexpr int kFusedTY = 8;   // float64 fused tiles: 32 x 8 nodes, one row per wave
// float32 / float16-shifted fused tiles: 64 x 4 nodes, one row of 64 per wave.
// Measured against 32 x 8: +2% (float32) and +14% (float16) at 256^3, +24%
// and +8% at 512^3 -- a float16 row of 64 is one whole 128-byte line, so
// fewer lines are written in part at the tile's x edges.
constexpr int kFloatTX = 64;
constexpr int kFloatTY = 4;
// Float storage without solids: 64 x 8 tiles, 16 waves at four per SIMD
// (128 registers), where their columns are marched in chunks of at least 64
// planes.  At 256^3 on the tile-major layout: float32 1.30 -> 1.12 ms with
// the layout change included (5.7% from the tiles alone in the structure of
// arrays), float16-shifted 0.84 -> 0.75 ms (in the structure of arrays they
// were 11% slower).  On 128^3 they would take 16-plane chunks (7% slower), so
// such lattices keep 64 x 4, as do lattices with solids (3% slower at 512^3).
constexpr int kFloatTallTY = 8;
constexpr int kFloatTallMinChunk = 64;
// Register prefetch depth of the float kernel: two planes ahead measured 2%
// (float32) and 1.5% (float16) faster than three at 256^3 (fewer registers,
// 133 against 152).
constexpr int kFloatDepth = 2;
// float32 without solids on the tile-major layout: loads issued two
// iterations before their plane's psi is published (LEAD = 2, 168
// registers, so 64 x 4 tiles at two waves per SIMD): 1.056 -> 0.985 ms at
// 256^3 against 64 x 8 tiles with one iteration of lead.  float16-shifted
// went the other way (0.729 -> 0.794 ms) and keeps the 64 x 8 tiles.
constexpr int kFloat32Lead = 2;
// Adjoint stencil march: columns in chunks of at least kAdjMarchMinChunk
// planes (each chunk re-reads the two planes beside it), enough chunks for
// kAdjMarchWGs workgroups per compute unit.  At 128^3 (8-plane chunks, four
// workgroups per CU) the backward pass took 189 instead of 192 ms (float32)
// and 398 instead of 410 ms (float64) against the per-node gather; 32-plane
// chunks, one workgroup per CU, made float32 slower (200 ms).
constexpr int kAdjMarchMinChunk = 8;
constexpr int kAdjMarchWGs = 4;
// Staged float64 step on 64 x 4 tiles (two waves per row) where nx allows:
// 9% faster than 32 x 8 at 256^3 -- half as many tile edges in x, where a
// push store writes a 128-byte line only in part.  The unstaged kernel was
// slower on 64 x 4 tiles and keeps 32 x 8.
constexpr int kWideTX = 64;
constexpr int kWideTY = 4;

constexpr int kTotalsMaxBlocks = 2048;
constexpr long long kSnapshotTotalsMaxNodes = 0x7fffffffLL - 4096;  // the 32-bit node index of the kernels

struct TimedLaunch {
  int slot;
  hipEvent_t start, stop;
};

}  // namespace

struct lb_ctx {
  lb_params p{};
  Geometry g{};
  StepCoeffs c{};
  size_t elem = 0;         // bytes per stored population value
  size_t real_bytes = 0;   // bytes of the arithmetic type
  size_t grid_bytes = 0;   // bytes of one population grid
  void* grid[2] = {nullptr, nullptr};
  int cur = 0;             // grid holding the current state
  void* psi = nullptr;     // [2][N] pseudopotential, arithmetic type
  uint8_t* mask = nullptr; // [N], allocated on first use
  bool has_solid = false;
  bool tiled = false;  // the current population grid is in the tile-major layout
  double* partial = nullptr;
  double* result = nullptr;
  int* flag = nullptr;
  double* plane = nullptr;  // [N] float64 staging for host transfers
  bool has_state = false;
  hipStream_t stream = nullptr;
  bool timing = false;
  std::vector<TimedLaunch> launches;
  std::vector<hipEvent_t> event_pool;
  double t_ms[SLOT_COUNT] = {};
  int64_t t_n[SLOT_COUNT] = {};
  // adjoint buffers, allocated by lb_adjoint_begin
  void* lam[2] = {nullptr, nullptr};  // [38][Npad] arithmetic type
  int lam_cur = 0;
  void* amom = nullptr;               // [10][N]
  void* wbuf = nullptr;               // [6][N]
  void* rbuf = nullptr;               // [2][N] stencil term of lam
  double* adj_partial = nullptr;      // per-block dJ/dG
  double* adj_dG = nullptr;           // running dJ/dG
  bool adj_ready = false;
  int kernel = LB_KERNEL_FUSED_STAGED;  // LB_KERNEL_AUTO
  int model = LB_MODEL_SHAN_CHEN;
  FusedTiling tiling{};       // the storage's default fused kernel
  FusedTiling tiling_wide{};  // staged float64 kernel on 64 x 4 tiles (nx a multiple of 64)
  FusedTiling tiling_cg{};    // float32 colour-gradient kernel (64 x 4 tiles)
  FusedTiling tiling_tall{};  // float Shan-Chen kernel without solids (64 x 8 tiles)
  bool tall = false;          // tiling_tall is used (its chunks hold >= kFloatTallMinChunk planes)
  FusedTiling tiling_adj{};   // z-marching adjoint stencil kernel (64 x 4 tiles)
  bool adj_march = false;     // k_adj_r_march runs the adjoint stencil term (nx % 64 == 0, ny % 4 == 0)
  int64_t bytes = 0;
  // moving particles (lb_set_particles, colour-gradient model)
  int np = 0;
  int part_cap = 0;            // particles the buffer below holds
  PartState ps{};
  double* part = nullptr;      // [5][P][3]: pos, vel, omg, force, torque
  int* owner[2] = {nullptr, nullptr};
  int ocur = 0;
  double* rho_buf = nullptr;   // [2][N] densities recorded near particles
};

namespace {

#define LB_HIP(call)                   \
  do {                                 \
    if ((call) != hipSuccess) {        \
      (void)hipGetLastError();         \
      return LB_EDEVICE;               \
    }                                  \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int blocks_for(long long n) { return static_cast<int>((n + kBlock - 1) / kBlock); }

// float16-shifted storage keeps f_i - w_i rho0_k; the other storages keep f.
void set_shift(const lb_params& p, StepCoeffs* c) {
  for (int k = 0; k < 2; ++k)
    for (int i = 0; i < Q; ++i)
      c->shift[k][i] = p.storage == LB_F16_SHIFTED ? static_cast<float>(weight<double>(i) * p.rho0[k]) : 0.0f;
}

lb_status dev_alloc(lb_ctx* ctx, void** ptr, size_t bytes) {
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return LB_ENOMEM;
  }
  ctx->bytes += static_cast<int64_t>(bytes);
  return LB_OK;
}

void free_all(lb_ctx* ctx) {
  if (ctx->stream != nullptr || true) (void)hipStreamSynchronize(ctx->stream);
  for (auto& l : ctx->launches) {
    (void)hipEventDestroy(l.start);
    (void)hipEventDestroy(l.stop);
  }
  ctx->launches.clear();
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  ctx->event_pool.clear();
  void* bufs[] = {ctx->grid[0], ctx->grid[1], ctx->psi,         ctx->mask,   ctx->partial,  ctx->result,
                  ctx->flag,    ctx->plane,   ctx->lam[0],      ctx->lam[1], ctx->amom,     ctx->wbuf,
                  ctx->rbuf,    ctx->adj_partial, ctx->adj_dG,  ctx->part,   ctx->owner[0], ctx->owner[1],
                  ctx->rho_buf};
  for (void* b : bufs)
    if (b != nullptr) (void)hipFree(b);
}

hipEvent_t take_event(lb_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Launch through `fn`, bracketing it with events when timing is on.
template <typename Fn>
lb_status launch(lb_ctx* ctx, int slot, Fn&& fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ctx->timing) {
    a = take_event(ctx);
    b = take_event(ctx);
    if (a == nullptr || b == nullptr) return LB_EDEVICE;
    LB_HIP(hipEventRecord(a, ctx->stream));
  }
  fn();
  LB_HIP(hipGetLastError());
  if (ctx->timing) {
    LB_HIP(hipEventRecord(b, ctx->stream));
    ctx->launches.push_back({slot, a, b});
  }
  return LB_OK;
}

lb_status fold_timing(lb_ctx* ctx) {
  if (ctx->launches.empty()) return LB_OK;
  LB_HIP(hipStreamSynchronize(ctx->stream));
  for (auto& l : ctx->launches) {
    float ms = 0.0f;
    LB_HIP(hipEventElapsedTime(&ms, l.start, l.stop));
    ctx->t_ms[l.slot] += ms;
    ctx->t_n[l.slot] += 1;
    ctx->event_pool.push_back(l.start);
    ctx->event_pool.push_back(l.stop);
  }
  ctx->launches.clear();
  return LB_OK;
}

bool is_finite(double v) { return std::isfinite(v); }

// mask of solid nodes (fixed solids or particles), or nullptr
const uint8_t* mask_or_null(const lb_ctx* ctx) { return (ctx->has_solid || ctx->np > 0) ? ctx->mask : nullptr; }

// ---------------------------------------------------------------------------
// Typed implementations
// ---------------------------------------------------------------------------
// One fused step from fin to fout.  float64: component-pair waves, either
// without prefetch or (LB_KERNEL_FUSED_STAGED, nx a multiple of 32, no
// solids) with the plane two ahead staged into LDS by direct-to-LDS loads,
// on 64 x 4 tiles when nx is a multiple of 64; float32 arithmetic:
// single-component waves with a register prefetch depth of three planes.  With rec != nullptr the kernel also writes the moment record of
// the pre-collision state for the adjoint.
bool staged_fits(const lb_ctx* ctx) { return ctx->p.storage == LB_F64 && ctx->p.nx % kFusedTX == 0; }
bool staged_wide(const lb_ctx* ctx) { return ctx->p.storage == LB_F64 && ctx->p.nx % kWideTX == 0; }

template <int ST, bool SOLID, bool RECORD>
void launch_fused_as(lb_ctx* ctx, const typename StorageTraits<ST>::store_t* fin,
                     typename StorageTraits<ST>::store_t* fout, typename StorageTraits<ST>::real* rec,
                     bool tiled = false) {
  const uint8_t* m = SOLID ? ctx->mask : nullptr;
  if constexpr (ST == ST_F64) {
    if constexpr (!SOLID) {
      if (tiled) {  // the caller has checked tiled_ok and put the grids in the tile-major layout
        const FusedTiling t = ctx->tiling_wide;
        k_fused_pair<ST, false, kWideTY, RECORD, true, kWideTX, kModelSC, true>
            <<<dim3(t.total), dim3(2 * kWideTX * kWideTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t,
                                                                               rec);
        return;
      }
    }
    if constexpr (!SOLID) {
      if (ctx->kernel == LB_KERNEL_FUSED_STAGED && staged_wide(ctx)) {
        const FusedTiling t = ctx->tiling_wide;
        k_fused_pair<ST, false, kWideTY, RECORD, true, kWideTX>
            <<<dim3(t.total), dim3(2 * kWideTX * kWideTY), 0, ctx->stream>>>(fin, fout, m, ctx->g, ctx->c, t, rec);
        return;
      }
      if (ctx->kernel == LB_KERNEL_FUSED_STAGED && staged_fits(ctx)) {
        const FusedTiling t = ctx->tiling;
        k_fused_pair<ST, false, kFusedTY, RECORD, true>
            <<<dim3(t.total), dim3(64 * kFusedTY), 0, ctx->stream>>>(fin, fout, m, ctx->g, ctx->c, t, rec);
        return;
      }
    }
    const FusedTiling t = ctx->tiling;
    k_fused_pair<ST, SOLID, kFusedTY, RECORD, false>
        <<<dim3(t.total), dim3(64 * kFusedTY), 0, ctx->stream>>>(fin, fout, m, ctx->g, ctx->c, t, rec);
  } else {
    if constexpr (SOLID) {
      if (tiled) {  // the caller has checked tiled_ok and put the grids in the tile-major layout
        const FusedTiling t = ctx->tiling;
        k_fused<ST, true, kFloatTY, kFloatDepth, RECORD, kFloatTX, true>
            <<<dim3(t.total), dim3(128 * kFloatTY * kFloatTX / 64), 0, ctx->stream>>>(fin, fout, m, ctx->g, ctx->c, t,
                                                                                       rec);
        return;
      }
    }
    if constexpr (!SOLID) {
      if (tiled) {  // the caller has checked tiled_ok and put the grids in the tile-major layout
        if constexpr (ST == ST_F32) {
          const FusedTiling t = ctx->tiling;
          k_fused<ST, false, kFloatTY, kFloatDepth, RECORD, kFloatTX, true, kFloat32Lead>
              <<<dim3(t.total), dim3(128 * kFloatTY * kFloatTX / 64), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g,
                                                                                         ctx->c, t, rec);
          return;
        }
        if (ctx->tall) {
          const FusedTiling t = ctx->tiling_tall;
          k_fused<ST, false, kFloatTallTY, kFloatDepth, RECORD, kFloatTX, true>
              <<<dim3(t.total), dim3(128 * kFloatTallTY * kFloatTX / 64), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g,
                                                                                             ctx->c, t, rec);
        } else {
          const FusedTiling t = ctx->tiling;
          k_fused<ST, false, kFloatTY, kFloatDepth, RECORD, kFloatTX, true>
              <<<dim3(t.total), dim3(128 * kFloatTY * kFloatTX / 64), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g,
                                                                                         ctx->c, t, rec);
        }
        return;
      }
    }
    if constexpr (ST == ST_F32 && !SOLID) {
      if (ctx->tall) {
        const FusedTiling t = ctx->tiling_tall;
        k_fused<ST, false, kFloatTallTY, kFloatDepth, RECORD, kFloatTX>
            <<<dim3(t.total), dim3(128 * kFloatTallTY * kFloatTX / 64), 0, ctx->stream>>>(fin, fout, m, ctx->g, ctx->c,
                                                                                           t, rec);
        return;
      }
    }
    const FusedTiling t = ctx->tiling;
    k_fused<ST, SOLID, kFloatTY, kFloatDepth, RECORD, kFloatTX>
        <<<dim3(t.total), dim3(128 * kFloatTY * kFloatTX / 64), 0, ctx->stream>>>(fin, fout, m, ctx->g, ctx->c, t, rec);
  }
}

// Colour-gradient step from fin to fout: the component-pair kernel with the
// colour-gradient collision.  float64 runs staged where the Shan-Chen step
// would (same tiles and tiling); float32 runs unstaged on 64 x 4 tiles (the
// float storages' tiling).
template <int ST>
void launch_cg_as(lb_ctx* ctx, const typename StorageTraits<ST>::store_t* fin,
                  typename StorageTraits<ST>::store_t* fout, bool tiled = false) {
  if constexpr (ST == ST_F64) {
    if (tiled) {  // the caller has checked tiled_ok and put the grids in the tile-major layout
      const FusedTiling t = ctx->tiling_wide;
      k_fused_pair<ST, false, kWideTY, false, true, kWideTX, kModelCG, true>
          <<<dim3(t.total), dim3(2 * kWideTX * kWideTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t,
                                                                             nullptr);
      return;
    }
    if (ctx->kernel == LB_KERNEL_FUSED_STAGED && staged_wide(ctx)) {
      const FusedTiling t = ctx->tiling_wide;
      k_fused_pair<ST, false, kWideTY, false, true, kWideTX, kModelCG>
          <<<dim3(t.total), dim3(2 * kWideTX * kWideTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t,
                                                                             nullptr);
      return;
    }
    const FusedTiling t = ctx->tiling;
    if (ctx->kernel == LB_KERNEL_FUSED_STAGED && staged_fits(ctx)) {
      k_fused_pair<ST, false, kFusedTY, false, true, kFusedTX, kModelCG>
          <<<dim3(t.total), dim3(64 * kFusedTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t, nullptr);
      return;
    }
    k_fused_pair<ST, false, kFusedTY, false, false, kFusedTX, kModelCG>
        <<<dim3(t.total), dim3(64 * kFusedTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t, nullptr);
  } else if constexpr (ST == ST_F32) {
    const FusedTiling t = ctx->tiling_cg;
    if (tiled) {  // the caller has checked tiled_ok and put the grids in the tile-major layout
      k_fused_pair<ST, false, kFloatTY, false, false, kFloatTX, kModelCG, true>
          <<<dim3(t.total), dim3(2 * kFloatTX * kFloatTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t,
                                                                               nullptr);
      return;
    }
    k_fused_pair<ST, false, kFloatTY, false, false, kFloatTX, kModelCG>
        <<<dim3(t.total), dim3(2 * kFloatTX * kFloatTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t,
                                                                             nullptr);
  }
}

template <int ST>
lb_status launch_fused(lb_ctx* ctx, const typename StorageTraits<ST>::store_t* fin,
                       typename StorageTraits<ST>::store_t* fout, typename StorageTraits<ST>::real* rec,
                       bool tiled = false) {
  if (ctx->model == LB_MODEL_COLOUR_GRADIENT) {
    // lb_set_model admits float64 and float32 storage without solids only
    if (ST == ST_F16S || ctx->has_solid || rec != nullptr) return LB_EINVAL;
    return launch(ctx, SLOT_FUSED, [&] { launch_cg_as<ST>(ctx, fin, fout, tiled); });
  }
  const bool solid = ctx->has_solid;
  return launch(ctx, SLOT_FUSED, [&] {
    if (solid) {
      if (rec) launch_fused_as<ST, true, true>(ctx, fin, fout, rec, tiled);
      else launch_fused_as<ST, true, false>(ctx, fin, fout, rec, tiled);
    } else {
      if (rec) launch_fused_as<ST, false, true>(ctx, fin, fout, rec, tiled);
      else launch_fused_as<ST, false, false>(ctx, fin, fout, rec, tiled);
    }
  });
}

// The fused steps run on the tile-major layout (one contiguous block per
// tile plane instead of 38 streams) where nx is a multiple of 64 and ny of 4:
// the staged float64 step without solids (either model) and every float
// step.
bool tiled_ok(const lb_ctx* ctx) {
  if (ctx->p.nx % kTileX != 0 || ctx->p.ny % kTileY != 0 || 2.0 * Q * ctx->g.nx * ctx->g.ny * ctx->elem >= 4294967296.0)
    return false;
  if (ctx->p.storage == LB_F64)  // the staged pair kernel; lattices with solids run the unstaged one
    return !ctx->has_solid && ctx->kernel == LB_KERNEL_FUSED_STAGED && staged_wide(ctx);
  return true;  // float storage: k_fused (Shan-Chen, with or without solids) or the pair kernel (colour gradient)
}

// Put the current grid in the tile-major (tiled) or the structure-of-arrays
// layout, through the other grid.  Every entry point other than the step
// asks for the structure-of-arrays layout before it touches the grid.
template <typename F>
lb_status by_storage(const lb_ctx* ctx, F&& f);

// Copy the grid at src into dst, from the tile-major layout (to_tiled = 0)
// or into it (1).
lb_status relayout(lb_ctx* ctx, const void* src, void* dst, int to_tiled) {
  return by_storage(ctx, [&](auto tag) {
    using store = typename StorageTraits<decltype(tag)::value>::store_t;
    k_relayout<store><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(static_cast<const store*>(src),
                                                                        static_cast<store*>(dst), ctx->g, to_tiled);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_EDEVICE;
  });
}

lb_status set_layout(lb_ctx* ctx, bool tiled) {
  if (ctx->tiled == tiled) return LB_OK;
  lb_status st = relayout(ctx, ctx->grid[ctx->cur], ctx->grid[ctx->cur ^ 1], tiled ? 1 : 0);
  if (st != LB_OK) return st;
  ctx->cur ^= 1;
  ctx->tiled = tiled;
  return LB_OK;
}

template <int ST>
lb_status fused_step_impl(lb_ctx* ctx, int n) {
  using store = typename StorageTraits<ST>::store_t;
  const bool tiled = tiled_ok(ctx);
  {
    lb_status st = set_layout(ctx, tiled);
    if (st != LB_OK) return st;
  }
  for (int s = 0; s < n; ++s) {
    const store* fin = static_cast<const store*>(ctx->grid[ctx->cur]);
    store* fout = static_cast<store*>(ctx->grid[ctx->cur ^ 1]);
    lb_status st = launch_fused<ST>(ctx, fin, fout, nullptr, tiled);
    if (st != LB_OK) return st;
    ctx->cur ^= 1;
  }
  return LB_OK;
}

// The fused kernels address a population plane with 32-bit byte offsets.
bool fused_fits(const lb_ctx* ctx) { return static_cast<double>(ctx->g.N) * ctx->elem < 4294967296.0; }
bool use_fused(const lb_ctx* ctx) {
  return (ctx->kernel == LB_KERNEL_FUSED || ctx->kernel == LB_KERNEL_FUSED_STAGED) && fused_fits(ctx);
}

// Colour-gradient step with moving particles, per step: the pair kernel
// with the particle coupling (blind push, densities near particles), the
// link pass with forces and leap-frog, the owner map of the new positions,
// covering and uncovering.  On the tile-major layout where nx is a multiple
// of 64 and ny of 4 (every kernel of the step addresses it), else the
// structure of arrays.
template <int ST>
lb_status particle_step_impl(lb_ctx* ctx, int n) {
  if constexpr (ST == ST_F16S) {
    return LB_EINVAL;  // lb_set_particles admits float64 and float32 storage only
  } else {
    using store = typename StorageTraits<ST>::store_t;
    // the tile-major layout where the plain steps use it (64 x 4 tiles)
    const bool tiled = ctx->p.nx % kTileX == 0 && ctx->p.ny % kTileY == 0 &&
                       2.0 * Q * ctx->g.nx * ctx->g.ny * ctx->elem < 4294967296.0 &&
                       (ST != ST_F64 || ctx->p.nx % kWideTX == 0);
    lb_status st = set_layout(ctx, tiled);
    if (st != LB_OK) return st;
    for (int s = 0; s < n; ++s) {
      const store* fin = static_cast<const store*>(ctx->grid[ctx->cur]);
      store* fout = static_cast<store*>(ctx->grid[ctx->cur ^ 1]);
      const int* own = ctx->owner[ctx->ocur];
      int* own_new = ctx->owner[ctx->ocur ^ 1];
      const PartFluid pf{own, ctx->rho_buf};
      st = launch(ctx, SLOT_FUSED, [&] {
        if constexpr (ST == ST_F64) {
          if (tiled) {
            const FusedTiling t = ctx->tiling_wide;
            k_fused_pair<ST, true, kWideTY, false, false, kWideTX, kModelCG, true, true>
                <<<dim3(t.total), dim3(2 * kWideTX * kWideTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t,
                                                                                   nullptr, pf);
          } else {
            const FusedTiling t = ctx->tiling;
            k_fused_pair<ST, true, kFusedTY, false, false, kFusedTX, kModelCG, false, true>
                <<<dim3(t.total), dim3(64 * kFusedTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c, t, nullptr,
                                                                          pf);
          }
        } else {
          const FusedTiling t = ctx->tiling_cg;
          if (tiled)
            k_fused_pair<ST, true, kFloatTY, false, false, kFloatTX, kModelCG, true, true>
                <<<dim3(t.total), dim3(2 * kFloatTX * kFloatTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c,
                                                                                     t, nullptr, pf);
          else
            k_fused_pair<ST, true, kFloatTY, false, false, kFloatTX, kModelCG, false, true>
                <<<dim3(t.total), dim3(2 * kFloatTX * kFloatTY), 0, ctx->stream>>>(fin, fout, nullptr, ctx->g, ctx->c,
                                                                                     t, nullptr, pf);
        }
      });
      if (st != LB_OK) return st;
      st = launch(ctx, SLOT_PART_FORCE, [&] {
        if (tiled)
          kp_force_move<ST, 2, true><<<ctx->np, kPartThreads, 0, ctx->stream>>>(fout, own, ctx->rho_buf, ctx->ps,
                                                                               ctx->g, ctx->c);
        else
          kp_force_move<ST, 2, false><<<ctx->np, kPartThreads, 0, ctx->stream>>>(fout, own, ctx->rho_buf, ctx->ps,
                                                                                ctx->g, ctx->c);
      });
      if (st != LB_OK) return st;
      st = launch(ctx, SLOT_PART_OWNER, [&] {
        kp_owner_fill<<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(own_new, ctx->g.N);
        kp_owner_scatter<<<ctx->np, kBlock, 0, ctx->stream>>>(own_new, ctx->ps, ctx->g);
      });
      if (st != LB_OK) return st;
      st = launch(ctx, SLOT_PART_REMAP, [&] {
        if (tiled)
          kp_remap<ST, 2, true><<<ctx->np, kPartThreads, 0, ctx->stream>>>(fout, own, own_new, ctx->mask, ctx->ps,
                                                                          ctx->g, ctx->c);
        else
          kp_remap<ST, 2, false><<<ctx->np, kPartThreads, 0, ctx->stream>>>(fout, own, own_new, ctx->mask, ctx->ps,
                                                                           ctx->g, ctx->c);
      });
      if (st != LB_OK) return st;
      ctx->cur ^= 1;
      ctx->ocur ^= 1;
    }
    return LB_OK;
  }
}

template <int ST>
lb_status step_impl(lb_ctx* ctx, int n) {
  if (ctx->np > 0) return particle_step_impl<ST>(ctx, n);
  if (use_fused(ctx)) return fused_step_impl<ST>(ctx, n);
  if (ctx->model != LB_MODEL_SHAN_CHEN) return LB_EINVAL;  // the colour-gradient step is fused only
  {
    lb_status st = set_layout(ctx, false);
    if (st != LB_OK) return st;
  }
  using store = typename StorageTraits<ST>::store_t;
  using real = typename StorageTraits<ST>::real;
  const int nb = blocks_for(ctx->g.N);
  real* psi = static_cast<real*>(ctx->psi);
  for (int s = 0; s < n; ++s) {
    const store* fin = static_cast<const store*>(ctx->grid[ctx->cur]);
    store* fout = static_cast<store*>(ctx->grid[ctx->cur ^ 1]);
    lb_status st;
    if (ctx->has_solid) {
      st = launch(ctx, SLOT_PSI, [&] {
        k_psi<ST, true><<<nb, kBlock, 0, ctx->stream>>>(fin, psi, ctx->mask, ctx->g, ctx->c);
      });
      if (st != LB_OK) return st;
      st = launch(ctx, SLOT_COLLIDE, [&] {
        k_collide_push<ST, true><<<nb, kBlock, 0, ctx->stream>>>(fin, fout, psi, ctx->mask, ctx->g, ctx->c);
      });
    } else {
      st = launch(ctx, SLOT_PSI, [&] {
        k_psi<ST, false><<<nb, kBlock, 0, ctx->stream>>>(fin, psi, nullptr, ctx->g, ctx->c);
      });
      if (st != LB_OK) return st;
      st = launch(ctx, SLOT_COLLIDE, [&] {
        k_collide_push<ST, false><<<nb, kBlock, 0, ctx->stream>>>(fin, fout, psi, nullptr, ctx->g, ctx->c);
      });
    }
    if (st != LB_OK) return st;
    ctx->cur ^= 1;
  }
  return LB_OK;
}

template <int ST>
lb_status init_impl(lb_ctx* ctx, const double* ra, const double* rb, const double* u) {
  using store = typename StorageTraits<ST>::store_t;
  LB_HIP(hipMemsetAsync(ctx->grid[ctx->cur ^ 1], 0, ctx->grid_bytes, ctx->stream));
  k_init<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(ra, rb, u, mask_or_null(ctx),
                                                               static_cast<store*>(ctx->grid[ctx->cur]), ctx->g, ctx->c);
  LB_HIP(hipGetLastError());
  return LB_OK;
}

template <int ST>
lb_status decode_impl(lb_ctx* ctx, int plane, double* out) {
  using store = typename StorageTraits<ST>::store_t;
  if (ctx->tiled)  // read in whichever layout the steps left the state
    k_decode_plane<ST, true><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
        static_cast<const store*>(ctx->grid[ctx->cur]), out, mask_or_null(ctx), plane, ctx->g, ctx->c);
  else
    k_decode_plane<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
        static_cast<const store*>(ctx->grid[ctx->cur]), out, mask_or_null(ctx), plane, ctx->g, ctx->c);
  LB_HIP(hipGetLastError());
  return LB_OK;
}

template <int ST>
lb_status encode_impl(lb_ctx* ctx, int plane, const double* in) {
  using store = typename StorageTraits<ST>::store_t;
  k_encode_plane<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
      in, static_cast<store*>(ctx->grid[ctx->cur]), mask_or_null(ctx), plane, ctx->g, ctx->c);
  LB_HIP(hipGetLastError());
  return LB_OK;
}

template <int ST>
lb_status moments_impl(lb_ctx* ctx, double* ra, double* rb, double* u) {
  using store = typename StorageTraits<ST>::store_t;
  using real = typename StorageTraits<ST>::real;
  const store* f = static_cast<const store*>(ctx->grid[ctx->cur]);
  real* psi = static_cast<real*>(ctx->psi);
  const int nb = blocks_for(ctx->g.N);
  // The colour-gradient velocity has no force term: with G = 0 the kernel's
  // (m_A + m_B + (F_A + F_B) / 2) / rho adds an exact zero.
  StepCoeffs c = ctx->c;
  if (ctx->model == LB_MODEL_COLOUR_GRADIENT) {
    c.G = 0.0;
    c.Gf = 0.0f;
  }
  // the state is read in whichever layout the steps left it
  if (mask_or_null(ctx) != nullptr) {
    if (ctx->tiled) {
      k_psi<ST, true, true><<<nb, kBlock, 0, ctx->stream>>>(f, psi, ctx->mask, ctx->g, c);
      k_moments<ST, true, true><<<nb, kBlock, 0, ctx->stream>>>(f, psi, ctx->mask, ra, rb, u, ctx->g, c);
    } else {
      k_psi<ST, true><<<nb, kBlock, 0, ctx->stream>>>(f, psi, ctx->mask, ctx->g, c);
      k_moments<ST, true><<<nb, kBlock, 0, ctx->stream>>>(f, psi, ctx->mask, ra, rb, u, ctx->g, c);
    }
  } else {
    if (ctx->tiled) {
      k_psi<ST, false, true><<<nb, kBlock, 0, ctx->stream>>>(f, psi, nullptr, ctx->g, c);
      k_moments<ST, false, true><<<nb, kBlock, 0, ctx->stream>>>(f, psi, nullptr, ra, rb, u, ctx->g, c);
    } else {
      k_psi<ST, false><<<nb, kBlock, 0, ctx->stream>>>(f, psi, nullptr, ctx->g, c);
      k_moments<ST, false><<<nb, kBlock, 0, ctx->stream>>>(f, psi, nullptr, ra, rb, u, ctx->g, c);
    }
  }
  LB_HIP(hipGetLastError());
  return LB_OK;
}

template <int ST>
lb_status totals_impl(lb_ctx* ctx, int blocks) {
  using store = typename StorageTraits<ST>::store_t;
  if (ctx->tiled)  // the state is read in whichever layout the steps left it
    k_totals_partial<ST, 2, true><<<blocks, kBlock, 0, ctx->stream>>>(static_cast<const store*>(ctx->grid[ctx->cur]),
                                                                     mask_or_null(ctx), ctx->g, ctx->c, ctx->partial);
  else
    k_totals_partial<ST><<<blocks, kBlock, 0, ctx->stream>>>(static_cast<const store*>(ctx->grid[ctx->cur]),
                                                            mask_or_null(ctx), ctx->g, ctx->c, ctx->partial);
  LB_HIP(hipGetLastError());
  k_totals_final<<<1, kBlock, 0, ctx->stream>>>(ctx->partial, blocks, ctx->result);
  LB_HIP(hipGetLastError());
  return LB_OK;
}

// One step from the raw state at fin to fout (both device, the context's layout).
template <int ST>
lb_status step_between_impl(lb_ctx* ctx, const void* fin, void* fout) {
  using store = typename StorageTraits<ST>::store_t;
  using real = typename StorageTraits<ST>::real;
  const store* a = static_cast<const store*>(fin);
  store* b = static_cast<store*>(fout);
  if (use_fused(ctx)) return launch_fused<ST>(ctx, a, b, nullptr);
  const int nb = blocks_for(ctx->g.N);
  real* psi = static_cast<real*>(ctx->psi);
  const uint8_t* m = mask_or_null(ctx);
  lb_status st = launch(ctx, SLOT_PSI, [&] {
    if (m) k_psi<ST, true><<<nb, kBlock, 0, ctx->stream>>>(a, psi, m, ctx->g, ctx->c);
    else k_psi<ST, false><<<nb, kBlock, 0, ctx->stream>>>(a, psi, nullptr, ctx->g, ctx->c);
  });
  if (st != LB_OK) return st;
  return launch(ctx, SLOT_COLLIDE, [&] {
    if (m) k_collide_push<ST, true><<<nb, kBlock, 0, ctx->stream>>>(a, b, psi, m, ctx->g, ctx->c);
    else k_collide_push<ST, false><<<nb, kBlock, 0, ctx->stream>>>(a, b, psi, nullptr, ctx->g, ctx->c);
  });
}

template <int ST>
lb_status adjoint_alloc(lb_ctx* ctx) {
  using real = typename StorageTraits<ST>::real;
  if (ctx->adj_ready) return LB_OK;
  const size_t N = static_cast<size_t>(ctx->g.N);
  const size_t lam_bytes = sizeof(real) * static_cast<size_t>(2 * Q) * static_cast<size_t>(ctx->g.Npad);
  lb_status st = LB_OK;
  for (int b = 0; b < 2 && st == LB_OK; ++b) st = dev_alloc(ctx, &ctx->lam[b], lam_bytes);
  if (st == LB_OK) st = dev_alloc(ctx, &ctx->amom, sizeof(real) * kAdjMom * N);
  if (st == LB_OK) st = dev_alloc(ctx, &ctx->wbuf, sizeof(real) * 6 * N);
  if (st == LB_OK) st = dev_alloc(ctx, &ctx->rbuf, sizeof(real) * 2 * N);
  if (st == LB_OK) st = dev_alloc(ctx, reinterpret_cast<void**>(&ctx->adj_partial), sizeof(double) * blocks_for(ctx->g.N));
  if (st == LB_OK) st = dev_alloc(ctx, reinterpret_cast<void**>(&ctx->adj_dG), sizeof(double) * 2);
  if (st != LB_OK) return st;
  // the padding of each plane is never written by the kernels; keep it zero
  LB_HIP(hipMemsetAsync(ctx->lam[0], 0, lam_bytes, ctx->stream));
  LB_HIP(hipMemsetAsync(ctx->lam[1], 0, lam_bytes, ctx->stream));
  ctx->adj_ready = true;
  return LB_OK;
}

template <int ST>
lb_status adjoint_begin_impl(lb_ctx* ctx, const double* ga, const double* gb) {
  using real = typename StorageTraits<ST>::real;
  lb_status st = adjoint_alloc<ST>(ctx);
  if (st != LB_OK) return st;
  ctx->lam_cur = 0;
  k_adj_seed<real><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
      ga, gb, mask_or_null(ctx), static_cast<real*>(ctx->lam[0]), static_cast<real*>(ctx->rbuf), ctx->g);
  LB_HIP(hipGetLastError());
  LB_HIP(hipMemsetAsync(ctx->adj_dG, 0, sizeof(double) * 2, ctx->stream));
  LB_HIP(hipMemsetAsync(ctx->adj_partial, 0, sizeof(double) * blocks_for(ctx->g.N), ctx->stream));
  return LB_OK;
}

// One adjoint step given the moment record of f(t) (rho, m, psi as [10][N]).
template <int ST>
lb_status adjoint_record_step_impl(lb_ctx* ctx, const typename StorageTraits<ST>::real* mom) {
  using real = typename StorageTraits<ST>::real;
  const int nb = blocks_for(ctx->g.N);
  const uint8_t* m = mask_or_null(ctx);
  real* W = static_cast<real*>(ctx->wbuf);
  real* r = static_cast<real*>(ctx->rbuf);
  const real* lin = static_cast<const real*>(ctx->lam[ctx->lam_cur]);
  real* lout = static_cast<real*>(ctx->lam[ctx->lam_cur ^ 1]);
  lb_status st = launch(ctx, SLOT_ADJ_LOCAL, [&] {
    k_adj_local<ST><<<nb, kBlock, 0, ctx->stream>>>(lin, r, lout, mom, m, W, ctx->adj_partial, ctx->g, ctx->c);
  });
  if (st != LB_OK) return st;
  st = launch(ctx, SLOT_ADJ_R, [&] {
    if (ctx->adj_march) {
      const FusedTiling t = ctx->tiling_adj;
      k_adj_r_march<ST><<<dim3(t.total), dim3(256), 0, ctx->stream>>>(mom, W, m, r, ctx->g, ctx->c, t);
    } else {
      k_adj_r<ST><<<nb, kBlock, 0, ctx->stream>>>(mom, W, m, r, ctx->g, ctx->c);
    }
  });
  if (st != LB_OK) return st;
  ctx->lam_cur ^= 1;
  return LB_OK;
}

// One adjoint step given a raw snapshot of f(t): moments first.
template <int ST>
lb_status adjoint_step_impl(lb_ctx* ctx, const void* state) {
  using store = typename StorageTraits<ST>::store_t;
  using real = typename StorageTraits<ST>::real;
  real* mom = static_cast<real*>(ctx->amom);
  lb_status st = launch(ctx, SLOT_ADJ_MOMENTS, [&] {
    k_adj_moments<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(static_cast<const store*>(state),
                                                                       mask_or_null(ctx), mom, ctx->g, ctx->c);
  });
  if (st != LB_OK) return st;
  return adjoint_record_step_impl<ST>(ctx, mom);
}

// One forward step of the context's state that also writes the moment record of f(t).
template <int ST>
lb_status step_record_impl(lb_ctx* ctx, void* record) {
  using store = typename StorageTraits<ST>::store_t;
  using real = typename StorageTraits<ST>::real;
  const store* fin = static_cast<const store*>(ctx->grid[ctx->cur]);
  store* fout = static_cast<store*>(ctx->grid[ctx->cur ^ 1]);
  real* rec = static_cast<real*>(record);
  lb_status st;
  if (use_fused(ctx)) {
    // the record step runs on the tile-major layout where the plain step
    // does (the record itself is indexed by node, whatever the layout)
    const bool tiled = tiled_ok(ctx);
    st = set_layout(ctx, tiled);
    if (st != LB_OK) return st;
    fin = static_cast<const store*>(ctx->grid[ctx->cur]);
    fout = static_cast<store*>(ctx->grid[ctx->cur ^ 1]);
    st = launch_fused<ST>(ctx, fin, fout, rec, tiled);
  } else {
    st = set_layout(ctx, false);
    if (st != LB_OK) return st;
    st = launch(ctx, SLOT_ADJ_MOMENTS, [&] {
      k_adj_moments<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(fin, mask_or_null(ctx), rec, ctx->g, ctx->c);
    });
    if (st == LB_OK) st = step_between_impl<ST>(ctx, fin, fout);
  }
  if (st != LB_OK) return st;
  ctx->cur ^= 1;
  return LB_OK;
}

template <int ST>
lb_status adjoint_result_impl(lb_ctx* ctx, double* ga, double* gb) {
  using real = typename StorageTraits<ST>::real;
  k_adj_result<real><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
      static_cast<const real*>(ctx->lam[ctx->lam_cur]), static_cast<const real*>(ctx->rbuf), ga, gb, ctx->g);
  LB_HIP(hipGetLastError());
  return LB_OK;
}

template <int ST>
lb_status adjoint_export_impl(lb_ctx* ctx, double* out) {
  using real = typename StorageTraits<ST>::real;
  k_adj_export<real><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
      static_cast<const real*>(ctx->lam[ctx->lam_cur]), static_cast<const real*>(ctx->rbuf), out, ctx->g);
  LB_HIP(hipGetLastError());
  return LB_OK;
}

template <typename F>
lb_status by_storage(const lb_ctx* ctx, F&& f) {
  switch (ctx->p.storage) {
    case LB_F64: return f(std::integral_constant<int, ST_F64>{});
    case LB_F32: return f(std::integral_constant<int, ST_F32>{});
    case LB_F16_SHIFTED: return f(std::integral_constant<int, ST_F16S>{});
    default: return LB_EINVAL;
  }
}

lb_status ensure_plane(lb_ctx* ctx) {
  if (ctx->plane != nullptr) return LB_OK;
  return dev_alloc(ctx, reinterpret_cast<void**>(&ctx->plane), sizeof(double) * static_cast<size_t>(ctx->g.N));
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// ---------------------------------------------------------------------------
// Single-fluid step (lb1_*): one population set, no force.
// ---------------------------------------------------------------------------
struct lb1_ctx {
  lb_params p{};
  Geometry g{};
  StepCoeffs c{};
  size_t elem = 0;
  size_t grid_bytes = 0;
  void* grid[2] = {nullptr, nullptr};
  int cur = 0;
  uint8_t* mask = nullptr;
  bool has_solid = false;
  double* partial = nullptr;
  double* result = nullptr;
  int* flag = nullptr;
  double* plane = nullptr;
  bool has_state = false;
  hipStream_t stream = nullptr;
  // moving particles (lb1_set_particles)
  int np = 0;
  int part_cap = 0;         // particles the buffer below holds
  PartState ps{};
  double* part = nullptr;   // [5][P][3]: pos, vel, omg, force, torque
  int* owner[2] = {nullptr, nullptr};
  int ocur = 0;
  double* rho_buf = nullptr;  // [N]
};

namespace {

template <typename F>
lb_status by_storage_id(int storage, F&& f) {
  switch (storage) {
    case LB_F64: return f(std::integral_constant<int, ST_F64>{});
    case LB_F32: return f(std::integral_constant<int, ST_F32>{});
    case LB_F16_SHIFTED: return f(std::integral_constant<int, ST_F16S>{});
    default: return LB_EINVAL;
  }
}

lb_status alloc1(void** ptr, size_t bytes) {
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return LB_ENOMEM;
  }
  return LB_OK;
}

// mask of solid nodes (fixed solids or particles), or nullptr
const uint8_t* solid_of(const lb1_ctx* ctx) { return (ctx->has_solid || ctx->np > 0) ? ctx->mask : nullptr; }

void free1(lb1_ctx* ctx) {
  (void)hipStreamSynchronize(ctx->stream);
  void* bufs[] = {ctx->grid[0], ctx->grid[1], ctx->mask,     ctx->partial,  ctx->result, ctx->flag,
                  ctx->plane,   ctx->part,    ctx->owner[0], ctx->owner[1], ctx->rho_buf};
  for (void* b : bufs)
    if (b != nullptr) (void)hipFree(b);
}

// Particle state of either context to host arrays (each may be NULL).
template <class Ctx>
lb_status get_particles_common(Ctx* ctx, double* pos, double* vel, double* omega, double* force, double* torque) {
  if (ctx->np == 0) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t P = static_cast<size_t>(ctx->np);
  double* outs[5] = {pos, vel, omega, force, torque};
  const double* srcs[5] = {ctx->ps.pos, ctx->ps.vel, ctx->ps.omg, ctx->ps.force, ctx->ps.torque};
  for (int k = 0; k < 5; ++k)
    if (outs[k] != nullptr)
      LB_HIP(hipMemcpyAsync(outs[k], srcs[k], sizeof(double) * 3 * P, hipMemcpyDeviceToHost, ctx->stream));
  LB_HIP(hipStreamSynchronize(ctx->stream));
  return LB_OK;
}

// Particles of either context, after the caller has checked what its
// context admits: NC = 1 for the single fluid, 2 for the colour-gradient
// pair (whose grid must be in the structure-of-arrays layout).  `alloc`
// allocates device memory owned by the context.
template <int NC, class Ctx, class Alloc>
lb_status set_particles_common(Ctx* ctx, int32_t count, double radius, double mass, const double* pos,
                               const double* vel, const double* omega, Alloc&& alloc) {
  auto release = [&]() -> lb_status {  // the current particles' nodes turn to fluid at rest
    if (ctx->np == 0) return LB_OK;
    DeviceGuard dg(ctx->p.device);
    if (!dg.ok) return LB_EDEVICE;
    lb_status st = by_storage_id(ctx->p.storage, [&](auto tag) {
      constexpr int ST = decltype(tag)::value;
      kp_release<ST, NC><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
          static_cast<typename StorageTraits<ST>::store_t*>(ctx->grid[ctx->cur]), ctx->mask, ctx->p.rho0[0],
          ctx->p.rho0[1], ctx->g, ctx->c);
      return hipGetLastError() == hipSuccess ? LB_OK : LB_EDEVICE;
    });
    if (st == LB_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = LB_EDEVICE;
    if (st == LB_OK) ctx->np = 0;
    return st;
  };
  if (count == 0) return release();
  if (!is_finite(radius) || !(radius > 0.0) || std::isnan(mass) || !(mass > 0.0)) return LB_EINVAL;
  const int box = static_cast<int>(std::floor(2.0 * radius)) + 4;
  if (box > ctx->g.nx || box > ctx->g.ny || box > ctx->g.nz) return LB_EINVAL;  // a particle's box must fit the lattice
  const double L[3] = {double(ctx->g.nx), double(ctx->g.ny), double(ctx->g.nz)};
  const size_t P = static_cast<size_t>(count);
  std::vector<double> host(15 * P, 0.0);
  for (size_t q = 0; q < P; ++q)
    for (int a = 0; a < 3; ++a) {
      const double r = pos[3 * q + a];
      const double v = vel ? vel[3 * q + a] : 0.0;
      const double w = omega ? omega[3 * q + a] : 0.0;
      if (!is_finite(r) || r < 0.0 || r >= L[a]) return LB_EINVAL;
      if (!is_finite(v) || !(std::fabs(v) < 0.5) || !is_finite(w)) return LB_EINVAL;  // under half a node per step
      host[3 * q + a] = r;
      host[3 * P + 3 * q + a] = v;
      host[6 * P + 3 * q + a] = w;
    }
  {
    lb_status st = release();
    if (st != LB_OK) return st;
  }
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  if (ctx->part != nullptr && ctx->part_cap < count) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->part);
    ctx->part = nullptr;
    ctx->part_cap = 0;
  }
  if (ctx->part == nullptr) {
    if (alloc(reinterpret_cast<void**>(&ctx->part), sizeof(double) * 15 * P) != LB_OK) return LB_ENOMEM;
    ctx->part_cap = count;
  }
  for (int b = 0; b < 2; ++b)
    if (ctx->owner[b] == nullptr && alloc(reinterpret_cast<void**>(&ctx->owner[b]), sizeof(int) * N) != LB_OK)
      return LB_ENOMEM;
  if (ctx->rho_buf == nullptr && alloc(reinterpret_cast<void**>(&ctx->rho_buf), sizeof(double) * NC * N) != LB_OK)
    return LB_ENOMEM;
  if (ctx->mask == nullptr && alloc(reinterpret_cast<void**>(&ctx->mask), N) != LB_OK) return LB_ENOMEM;
  PartState& ps = ctx->ps;
  ps.pos = ctx->part;
  ps.vel = ctx->part + 3 * P;
  ps.omg = ctx->part + 6 * P;
  ps.force = ctx->part + 9 * P;
  ps.torque = ctx->part + 12 * P;
  ps.count = count;
  ps.box = box;
  ps.radius = radius;
  ps.r2 = radius * radius;
  ps.near2 = (radius + 1.5) * (radius + 1.5);
  ps.inner2 = radius > 1.5 ? (radius - 1.5) * (radius - 1.5) : -1.0;
  ps.mass = mass;
  ps.inertia = 0.4 * mass * radius * radius;
  ps.rho0[0] = ctx->p.rho0[0];
  ps.rho0[1] = NC == 2 ? ctx->p.rho0[1] : ctx->p.rho0[0];
  LB_HIP(hipMemcpyAsync(ctx->part, host.data(), sizeof(double) * 15 * P, hipMemcpyHostToDevice, ctx->stream));
  ctx->ocur = 0;
  kp_owner_fill<<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(ctx->owner[0], ctx->g.N);
  kp_owner_scatter<<<count, kBlock, 0, ctx->stream>>>(ctx->owner[0], ps, ctx->g);
  lb_status st = by_storage_id(ctx->p.storage, [&](auto tag) {
    constexpr int ST = decltype(tag)::value;
    kp_apply_owner<ST, NC><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
        static_cast<typename StorageTraits<ST>::store_t*>(ctx->grid[ctx->cur]), ctx->owner[0], ctx->mask, ctx->g);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_EDEVICE;
  });
  if (st != LB_OK) return st;
  LB_HIP(hipStreamSynchronize(ctx->stream));
  ctx->np = count;
  return LB_OK;
}


}  // namespace

// ---------------------------------------------------------------------------
// Device scratch of lb_snapshot_totals, the entry point that allocates
// nothing: kTotalsMaxBlocks per-workgroup partial sums of eight doubles,
// then eight result doubles (131,136 bytes).  Every device the library runs
// it on holds its own copy until the process ends.  Host code never uses the
// array's name as an address (on the host it names a stand-in, not device
// memory): the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kTotalsMaxBlocks * 8 + 8];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch[kScratchDevices] = {};

// Device address of `scratch` on `device`, which must be current.
lb_status scratch_address(int device, double** out) {
  if (device < 0 || device >= kScratchDevices) return LB_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch[device] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return LB_EDEVICE;
    }
    g_scratch[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch[device];
  return LB_OK;
}

template <int ST>
void snapshot_totals_launch(const void* f, const uint8_t* solid, const Geometry& g, const StepCoeffs& c, int blocks,
                            double* partial, double* result, hipStream_t stream) {
  using store = typename StorageTraits<ST>::store_t;
  k_totals_partial<ST><<<blocks, kBlock, 0, stream>>>(static_cast<const store*>(f), solid, g, c, partial);
  k_totals_final<<<1, kBlock, 0, stream>>>(partial, blocks, result);
}

}  // namespace

extern "C" {

lb_status lb_snapshot_totals(const lb_params* params, const void* snapshot, const uint8_t* solid, double* out,
                             int32_t on_device) {
  if (params == nullptr || snapshot == nullptr || out == nullptr) return LB_EINVAL;
  const lb_params& p = *params;
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return LB_EINVAL;
  if (p.storage != LB_F64 && p.storage != LB_F32 && p.storage != LB_F16_SHIFTED) return LB_EINVAL;
  if (p.storage == LB_F16_SHIFTED && !(is_finite(p.rho0[0]) && is_finite(p.rho0[1]))) return LB_EINVAL;
  const long long N = static_cast<long long>(p.nx) * p.ny * p.nz;
  if (N > kSnapshotTotalsMaxNodes) return LB_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) {
    (void)hipGetLastError();
    return LB_EDEVICE;
  }
  if (p.device < 0 || p.device >= ndev) return LB_EDEVICE;
  DeviceGuard dg(p.device);
  if (!dg.ok) return LB_EDEVICE;
  double* scr = nullptr;
  {
    const lb_status st = scratch_address(p.device, &scr);
    if (st != LB_OK) return st;
  }
  Geometry g{};
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.N = static_cast<int>(N);
  g.Npad = (N + 127) / 128 * 128;
  StepCoeffs c{};
  set_shift(p, &c);
  int blocks = blocks_for(N);
  if (blocks > kTotalsMaxBlocks) blocks = kTotalsMaxBlocks;
  double* partial = scr;                           // [blocks][8], each written before it is read
  double* result = scr + kTotalsMaxBlocks * 8;     // host results pass through here
  hipStream_t stream = static_cast<hipStream_t>(p.stream);
  double* dst = on_device ? out : result;
  if (p.storage == LB_F64) snapshot_totals_launch<LB_F64>(snapshot, solid, g, c, blocks, partial, dst, stream);
  else if (p.storage == LB_F32) snapshot_totals_launch<LB_F32>(snapshot, solid, g, c, blocks, partial, dst, stream);
  else snapshot_totals_launch<LB_F16_SHIFTED>(snapshot, solid, g, c, blocks, partial, dst, stream);
  LB_HIP(hipGetLastError());
  if (on_device) return LB_OK;
  LB_HIP(hipMemcpyAsync(out, result, sizeof(double) * kTotals, hipMemcpyDeviceToHost, stream));
  LB_HIP(hipStreamSynchronize(stream));
  return out[5] != 0.0 ? LB_ENONFINITE : LB_OK;
}

void lb_params_default(lb_params* p) {
  if (p == nullptr) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 1;
  p->tau[0] = p->tau[1] = 1.0;
  p->G = 0.0;
  p->psi_ref = 1.0;
  p->rho0[0] = p->rho0[1] = 1.0;
  p->storage = LB_F64;
  p->device = 0;
  p->stream = nullptr;
}

int32_t lb_abi_version(void) { return LB_ABI_VERSION; }

const char* lb_strerror(lb_status s) {
  switch (s) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument";
    case LB_ENOMEM: return "device allocation failed";
    case LB_EDEVICE: return "HIP runtime error or no usable device";
    case LB_ESTATE: return "no state set yet (call lb_set_fields or lb_set_populations first)";
    case LB_ENONFINITE: return "state holds NaN or Inf";
  }
  return "unknown status";
}

int32_t lb_timing_slots(void) { return SLOT_COUNT; }

const char* lb_timing_name(int32_t slot) {
  if (slot < 0 || slot >= SLOT_COUNT) return nullptr;
  return kSlotNames[slot];
}

// Fused-kernel tiling: columns of tile_x x tile_y nodes.  When the columns
// fit in one round of resident workgroups, z is split only as far as needed
// to give every compute unit a workgroup: each chunk end re-reads the plane
// beyond it and restarts the pipeline.  On 256^3 (256 columns of 64 x 4
// nodes, one per compute unit) whole columns beat four 64-plane chunks by
// 1.5% (float32) and 3.5% (float16) and tie for float64.  Lattices that take
// several rounds anyway use 64-plane chunks: on 512^3 (float32 and float16)
// they ran 22% faster than whole 512-plane columns.
// chunk_full_round: also use 64-plane chunks when the columns fill exactly
// one round (the unstaged component-pair kernel of the float32 colour-gradient
// step runs 17% faster so at 256^3).  min_chunk: the shortest chunk (or the
// whole column where it is shorter).
bool make_tiling(const lb_params& p, int tile_x, int tile_y, int cus, FusedTiling* out,
                 bool chunk_full_round = false, int min_chunk = 4) {
  FusedTiling t{};
  t.tiles_x = (p.nx + tile_x - 1) / tile_x;
  t.tiles_y = (p.ny + tile_y - 1) / tile_y;
  const long long cols = static_cast<long long>(t.tiles_x) * t.tiles_y;
  const long long target = cus;
  long long want = (target + cols - 1) / cols;  // chunks wanted
  if (cols > target || (chunk_full_round && cols == target)) want = p.nz / 64;
  if (want < 1) want = 1;
  int chunk = static_cast<int>((p.nz + want - 1) / want);
  if (chunk < min_chunk) chunk = min_chunk;
  if (chunk > p.nz) chunk = p.nz;
  t.chunk = chunk;
  t.chunks = (p.nz + chunk - 1) / chunk;
  const long long total = cols * t.chunks;
  if (total > 0x7fffffffLL) return false;
  t.total = static_cast<int>(total);
  // every fused kernel runs one workgroup per compute unit (register or
  // LDS bound), so a round of resident workgroups is one per unit
  t.per_round = ((cus + kXCDs - 1) / kXCDs) * kXCDs;
  *out = t;
  return true;
}

lb_status lb_create(const lb_params* params, lb_ctx** out) {
  if (out == nullptr) return LB_EINVAL;
  *out = nullptr;
  if (params == nullptr) return LB_EINVAL;
  const lb_params& p = *params;
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return LB_EINVAL;
  for (int k = 0; k < 2; ++k) {
    if (!is_finite(p.tau[k]) || !(p.tau[k] > 0.5)) return LB_EINVAL;
    if (!is_finite(p.rho0[k])) return LB_EINVAL;
  }
  if (!is_finite(p.G) || !is_finite(p.psi_ref) || !(p.psi_ref > 0.0)) return LB_EINVAL;
  if (p.storage != LB_F64 && p.storage != LB_F32 && p.storage != LB_F16_SHIFTED) return LB_EINVAL;
  const long long N = static_cast<long long>(p.nx) * p.ny * p.nz;
  if (N > 0x7fffffffLL - 4096) return LB_EINVAL;  // node index is 32-bit inside the kernels

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) {
    (void)hipGetLastError();
    return LB_EDEVICE;
  }
  if (p.device < 0 || p.device >= ndev) return LB_EDEVICE;
  DeviceGuard dg(p.device);
  if (!dg.ok) return LB_EDEVICE;

  lb_ctx* ctx = new (std::nothrow) lb_ctx();
  if (ctx == nullptr) return LB_ENOMEM;
  ctx->p = p;
  ctx->stream = static_cast<hipStream_t>(p.stream);
  ctx->g.nx = p.nx;
  ctx->g.ny = p.ny;
  ctx->g.nz = p.nz;
  ctx->g.N = static_cast<int>(N);
  ctx->g.Npad = (N + 127) / 128 * 128;  // keeps every plane 256-byte aligned
  ctx->elem = p.storage == LB_F64 ? 8 : (p.storage == LB_F32 ? 4 : 2);
  ctx->real_bytes = p.storage == LB_F64 ? 8 : 4;
  ctx->grid_bytes = ctx->elem * static_cast<size_t>(2 * Q) * static_cast<size_t>(ctx->g.Npad);

  StepCoeffs& c = ctx->c;
  for (int k = 0; k < 2; ++k) {
    c.om[k] = 1.0 / p.tau[k];
    c.omc[k] = 1.0 - c.om[k];
    c.tg[k] = p.tau[k] * p.G;
    c.tau[k] = p.tau[k];
    c.tauf[k] = static_cast<float>(p.tau[k]);
    c.omf[k] = static_cast<float>(c.om[k]);
    c.omcf[k] = static_cast<float>(c.omc[k]);
    c.tgf[k] = static_cast<float>(c.tg[k]);
  }
  set_shift(p, &c);
  c.G = p.G;
  c.psi_ref = p.psi_ref;

  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p.device) != hipSuccess || cus < 1)
      cus = 256;
    const bool f64 = p.storage == LB_F64;
    bool ok = make_tiling(p, f64 ? kFusedTX : kFloatTX, f64 ? kFusedTY : kFloatTY, cus, &ctx->tiling);
    if (ok && f64 && p.nx % kWideTX == 0) ok = make_tiling(p, kWideTX, kWideTY, cus, &ctx->tiling_wide);
    if (ok && !f64) ok = make_tiling(p, kFloatTX, kFloatTY, cus, &ctx->tiling_cg, true);
    if (ok && !f64) {
      ok = make_tiling(p, kFloatTX, kFloatTallTY, cus, &ctx->tiling_tall);
      ctx->tall = ok && ctx->tiling_tall.chunk >= kFloatTallMinChunk;
    }
    if (!ok) {
      delete ctx;
      return LB_EINVAL;
    }
    if (p.nx % kTileX == 0 && p.ny % kTileY == 0)
      ctx->adj_march = make_tiling(p, kTileX, kTileY, kAdjMarchWGs * cus, &ctx->tiling_adj, false, kAdjMarchMinChunk);
  }
  c.Gf = static_cast<float>(p.G);
  c.psi_reff = static_cast<float>(p.psi_ref);

  lb_status st = LB_OK;
  for (int b = 0; b < 2 && st == LB_OK; ++b) st = dev_alloc(ctx, &ctx->grid[b], ctx->grid_bytes);
  if (st == LB_OK) st = dev_alloc(ctx, &ctx->psi, ctx->real_bytes * 2 * static_cast<size_t>(N));
  if (st == LB_OK) st = dev_alloc(ctx, reinterpret_cast<void**>(&ctx->partial), sizeof(double) * 8 * kTotalsMaxBlocks);
  if (st == LB_OK) st = dev_alloc(ctx, reinterpret_cast<void**>(&ctx->result), sizeof(double) * 8);
  if (st == LB_OK) st = dev_alloc(ctx, reinterpret_cast<void**>(&ctx->flag), sizeof(int) * 4);
  if (st != LB_OK) {
    free_all(ctx);
    delete ctx;
    return st;
  }
  *out = ctx;
  return LB_OK;
}

lb_status lb_destroy(lb_ctx* ctx) {
  if (ctx == nullptr) return LB_OK;
  DeviceGuard dg(ctx->p.device);
  free_all(ctx);
  delete ctx;
  return LB_OK;
}

lb_status lb_set_stream(lb_ctx* ctx, void* stream) {
  if (ctx == nullptr) return LB_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  ctx->p.stream = stream;
  return LB_OK;
}

lb_status lb_set_kernel(lb_ctx* ctx, int32_t kernel) {
  if (ctx == nullptr) return LB_EINVAL;
  if (kernel == LB_KERNEL_AUTO) kernel = LB_KERNEL_FUSED_STAGED;  // runs as LB_KERNEL_FUSED where it does not apply
  if (kernel != LB_KERNEL_FUSED && kernel != LB_KERNEL_TWO_PASS && kernel != LB_KERNEL_FUSED_STAGED) return LB_EINVAL;
  ctx->kernel = kernel;
  return LB_OK;
}

lb_status lb_device_bytes(const lb_ctx* ctx, int64_t* bytes) {
  if (ctx == nullptr || bytes == nullptr) return LB_EINVAL;
  *bytes = ctx->bytes;
  return LB_OK;
}

lb_status lb_set_fields(lb_ctx* ctx, const double* rho_a, const double* rho_b, const double* u,
                        const uint8_t* solid, int on_device) {
  if (ctx == nullptr || rho_a == nullptr || rho_b == nullptr) return LB_EINVAL;
  if (solid != nullptr && ctx->model != LB_MODEL_SHAN_CHEN) return LB_EINVAL;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  const double* dra = rho_a;
  const double* drb = rho_b;
  const double* du = u;
  void* tmp = nullptr;
  if (!on_device) {
    const size_t n_in = (u != nullptr ? 5 : 2) * N;
    if (hipMalloc(&tmp, sizeof(double) * n_in) != hipSuccess) {
      (void)hipGetLastError();
      return LB_ENOMEM;
    }
    double* t = static_cast<double*>(tmp);
    bool ok = hipMemcpyAsync(t, rho_a, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream) == hipSuccess &&
              hipMemcpyAsync(t + N, rho_b, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
    if (ok && u != nullptr)
      ok = hipMemcpyAsync(t + 2 * N, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      (void)hipFree(tmp);
      return LB_EDEVICE;
    }
    dra = t;
    drb = t + N;
    du = u != nullptr ? t + 2 * N : nullptr;
  }
  auto release = [&]() {
    if (tmp != nullptr) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(tmp);
    }
  };
  // validate before touching the state
  int bad = 0;
  if (hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream) != hipSuccess) {
    release();
    return LB_EDEVICE;
  }
  k_validate_fields<<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(dra, drb, du, ctx->g.N, ctx->flag,
                                                                      ctx->model == LB_MODEL_COLOUR_GRADIENT);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&bad, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    release();
    return LB_EDEVICE;
  }
  if (bad) {
    release();
    return LB_EINVAL;
  }
  if (solid != nullptr) {
    if (ctx->mask == nullptr) {
      lb_status st = dev_alloc(ctx, reinterpret_cast<void**>(&ctx->mask), N);
      if (st != LB_OK) {
        release();
        return st;
      }
    }
    if (hipMemcpyAsync(ctx->mask, solid, N, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       ctx->stream) != hipSuccess) {
      (void)hipGetLastError();
      release();
      return LB_EDEVICE;
    }
    ctx->has_solid = true;
  } else {
    ctx->has_solid = false;
  }
  ctx->np = 0;  // new fields drop the particles
  lb_status st = by_storage(ctx, [&](auto tag) { return init_impl<decltype(tag)::value>(ctx, dra, drb, du); });
  if (st == LB_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = LB_EDEVICE;
  release();
  ctx->tiled = false;  // the initial state is written in the structure-of-arrays layout
  if (st == LB_OK) ctx->has_state = true;
  return st;
}

lb_status lb_step(lb_ctx* ctx, int32_t n) {
  if (ctx == nullptr || n < 0) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  if (n == 0) return LB_OK;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  return by_storage(ctx, [&](auto tag) { return step_impl<decltype(tag)::value>(ctx, n); });
}

lb_status lb_moments(lb_ctx* ctx, double* rho_a, double* rho_b, double* u, int on_device) {
  if (ctx == nullptr) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  // moments and totals read the state in either layout, so a read between steps reorders nothing
  const size_t N = static_cast<size_t>(ctx->g.N);
  if (on_device) {
    lb_status st = by_storage(ctx, [&](auto tag) { return moments_impl<decltype(tag)::value>(ctx, rho_a, rho_b, u); });
    if (st != LB_OK) return st;
    LB_HIP(hipStreamSynchronize(ctx->stream));
    return LB_OK;
  }
  void* tmp = nullptr;
  if (hipMalloc(&tmp, sizeof(double) * 5 * N) != hipSuccess) {
    (void)hipGetLastError();
    return LB_ENOMEM;
  }
  double* t = static_cast<double*>(tmp);
  lb_status st = by_storage(ctx, [&](auto tag) {
    return moments_impl<decltype(tag)::value>(ctx, rho_a ? t : nullptr, rho_b ? t + N : nullptr, u ? t + 2 * N : nullptr);
  });
  bool ok = st == LB_OK;
  if (ok && rho_a) ok = hipMemcpyAsync(rho_a, t, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
  if (ok && rho_b) ok = hipMemcpyAsync(rho_b, t + N, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
  if (ok && u) ok = hipMemcpyAsync(u, t + 2 * N, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(ctx->stream) == hipSuccess;
  (void)hipGetLastError();
  (void)hipFree(tmp);
  if (st != LB_OK) return st;
  return ok ? LB_OK : LB_EDEVICE;
}

lb_status lb_get_populations(lb_ctx* ctx, double* f, int on_device) {
  if (ctx == nullptr || f == nullptr) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  if (!on_device) {
    lb_status st = ensure_plane(ctx);
    if (st != LB_OK) return st;
  }
  for (int plane = 0; plane < 2 * Q; ++plane) {
    double* dst = on_device ? f + plane * N : ctx->plane;
    lb_status st = by_storage(ctx, [&](auto tag) { return decode_impl<decltype(tag)::value>(ctx, plane, dst); });
    if (st != LB_OK) return st;
    if (!on_device) {
      LB_HIP(hipMemcpyAsync(f + plane * N, ctx->plane, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
      LB_HIP(hipStreamSynchronize(ctx->stream));
    }
  }
  LB_HIP(hipStreamSynchronize(ctx->stream));
  return LB_OK;
}

lb_status lb_set_populations(lb_ctx* ctx, const double* f, int on_device) {
  if (ctx == nullptr || f == nullptr) return LB_EINVAL;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  lb_status st = ensure_plane(ctx);
  if (st != LB_OK) return st;
  // Reject non-finite input before anything is overwritten.
  LB_HIP(hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream));
  for (int plane = 0; plane < 2 * Q; ++plane) {
    const double* src = f + plane * N;
    if (!on_device) {
      LB_HIP(hipMemcpyAsync(ctx->plane, src, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
      src = ctx->plane;
    }
    k_check_finite<<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(src, ctx->g.N, ctx->flag);
    LB_HIP(hipGetLastError());
  }
  int bad = 0;
  LB_HIP(hipMemcpyAsync(&bad, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  LB_HIP(hipStreamSynchronize(ctx->stream));
  if (bad) return LB_EINVAL;
  if (!ctx->has_state) LB_HIP(hipMemsetAsync(ctx->grid[ctx->cur ^ 1], 0, ctx->grid_bytes, ctx->stream));
  ctx->tiled = false;  // every plane is written below, in the structure of arrays: the old state needs no reorder
  for (int plane = 0; plane < 2 * Q; ++plane) {
    const double* src = f + plane * N;
    if (!on_device) {
      LB_HIP(hipMemcpyAsync(ctx->plane, src, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
      src = ctx->plane;
    }
    st = by_storage(ctx, [&](auto tag) { return encode_impl<decltype(tag)::value>(ctx, plane, src); });
    if (st != LB_OK) return st;
  }
  LB_HIP(hipStreamSynchronize(ctx->stream));
  ctx->has_state = true;
  return LB_OK;
}

lb_status lb_totals(lb_ctx* ctx, double out[5], int* nonfinite) {
  if (ctx == nullptr || out == nullptr) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  int blocks = blocks_for(ctx->g.N);
  if (blocks > kTotalsMaxBlocks) blocks = kTotalsMaxBlocks;
  lb_status st = by_storage(ctx, [&](auto tag) { return totals_impl<decltype(tag)::value>(ctx, blocks); });
  if (st != LB_OK) return st;
  double r[8] = {0};
  LB_HIP(hipMemcpyAsync(r, ctx->result, sizeof(double) * kTotals, hipMemcpyDeviceToHost, ctx->stream));
  LB_HIP(hipStreamSynchronize(ctx->stream));
  for (int j = 0; j < 5; ++j) out[j] = r[j];
  const int nf = r[5] != 0.0 ? 1 : 0;
  if (nonfinite != nullptr) *nonfinite = nf;
  return nf ? LB_ENONFINITE : LB_OK;
}

lb_status lb_set_model(lb_ctx* ctx, int32_t model, double sigma, double beta) {
  if (ctx == nullptr) return LB_EINVAL;
  if (model != LB_MODEL_SHAN_CHEN && model != LB_MODEL_COLOUR_GRADIENT) return LB_EINVAL;
  if (!is_finite(sigma) || !is_finite(beta) || sigma < 0.0 || beta < 0.0) return LB_EINVAL;
  if (model == LB_MODEL_COLOUR_GRADIENT && (ctx->p.storage == LB_F16_SHIFTED || ctx->has_solid)) return LB_EINVAL;
  if (model != LB_MODEL_COLOUR_GRADIENT && ctx->np > 0) return LB_EINVAL;  // particles live in the colour-gradient fluid
  StepCoeffs& c = ctx->c;
  for (int k = 0; k < 2; ++k) {
    c.cg_inv_nu[k] = 1.0 / ((ctx->p.tau[k] - 0.5) / 3.0);
    c.cg_inv_nuf[k] = static_cast<float>(c.cg_inv_nu[k]);
  }
  c.cg_s225 = 2.25 * sigma;
  c.cg_beta = beta;
  c.cg_s225f = static_cast<float>(c.cg_s225);
  c.cg_betaf = static_cast<float>(beta);
  ctx->model = model;
  return LB_OK;
}

lb_status lb_set_coupling(lb_ctx* ctx, double G) {
  if (ctx == nullptr || !is_finite(G)) return LB_EINVAL;
  ctx->p.G = G;
  ctx->c.G = G;
  ctx->c.Gf = static_cast<float>(G);
  for (int k = 0; k < 2; ++k) {
    ctx->c.tg[k] = ctx->p.tau[k] * G;
    ctx->c.tgf[k] = static_cast<float>(ctx->c.tg[k]);
  }
  return LB_OK;
}

lb_status lb_state_bytes(const lb_ctx* ctx, int64_t* bytes) {
  if (ctx == nullptr || bytes == nullptr) return LB_EINVAL;
  *bytes = static_cast<int64_t>(ctx->grid_bytes);
  return LB_OK;
}

lb_status lb_save_state(lb_ctx* ctx, void* dst, int on_device) {
  if (ctx == nullptr || dst == nullptr) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  if (on_device && ctx->tiled) {  // the snapshot in the structure-of-arrays layout; the state stays as it is
    lb_status st = relayout(ctx, ctx->grid[ctx->cur], dst, 0);
    if (st != LB_OK) return st;
    LB_HIP(hipStreamSynchronize(ctx->stream));
    return LB_OK;
  }
  {
    lb_status lst = set_layout(ctx, false);  // the structure-of-arrays layout for everything but the step
    if (lst != LB_OK) return lst;
  }
  LB_HIP(hipMemcpyAsync(dst, ctx->grid[ctx->cur], ctx->grid_bytes,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
  LB_HIP(hipStreamSynchronize(ctx->stream));
  return LB_OK;
}

lb_status lb_restore_state(lb_ctx* ctx, const void* src, int on_device) {
  if (ctx == nullptr || src == nullptr) return LB_EINVAL;
  if (ctx->np > 0) return LB_EINVAL;  // a snapshot holds no particle state
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  if (!ctx->has_state) LB_HIP(hipMemsetAsync(ctx->grid[ctx->cur ^ 1], 0, ctx->grid_bytes, ctx->stream));
  LB_HIP(hipMemcpyAsync(ctx->grid[ctx->cur], src, ctx->grid_bytes,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
  LB_HIP(hipStreamSynchronize(ctx->stream));
  ctx->has_state = true;
  ctx->tiled = false;  // snapshots are in the structure-of-arrays layout
  return LB_OK;
}

lb_status lb_step_between(lb_ctx* ctx, const void* fin, void* fout) {
  if (ctx == nullptr || fin == nullptr || fout == nullptr || fin == fout) return LB_EINVAL;
  if (ctx->model != LB_MODEL_SHAN_CHEN) return LB_EINVAL;  // Shan-Chen only
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  return by_storage(ctx, [&](auto tag) { return step_between_impl<decltype(tag)::value>(ctx, fin, fout); });
}

lb_status lb_record_bytes(const lb_ctx* ctx, int64_t* bytes) {
  if (ctx == nullptr || bytes == nullptr) return LB_EINVAL;
  *bytes = static_cast<int64_t>(ctx->real_bytes) * kAdjMom * static_cast<int64_t>(ctx->g.N);
  return LB_OK;
}

lb_status lb_step_record(lb_ctx* ctx, void* record) {
  if (ctx == nullptr || record == nullptr) return LB_EINVAL;
  if (ctx->model != LB_MODEL_SHAN_CHEN) return LB_EINVAL;  // Shan-Chen only
  if (!ctx->has_state) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  return by_storage(ctx, [&](auto tag) { return step_record_impl<decltype(tag)::value>(ctx, record); });
}

lb_status lb_adjoint_step_record(lb_ctx* ctx, const void* record) {
  if (ctx == nullptr || record == nullptr) return LB_EINVAL;
  if (ctx->model != LB_MODEL_SHAN_CHEN) return LB_EINVAL;  // Shan-Chen only
  if (!ctx->adj_ready) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  return by_storage(ctx, [&](auto tag) {
    using real = typename StorageTraits<decltype(tag)::value>::real;
    return adjoint_record_step_impl<decltype(tag)::value>(ctx, static_cast<const real*>(record));
  });
}

lb_status lb_adjoint_begin(lb_ctx* ctx, const double* dJ_drho_a, const double* dJ_drho_b, int on_device) {
  if (ctx == nullptr) return LB_EINVAL;
  if (ctx->model != LB_MODEL_SHAN_CHEN) return LB_EINVAL;  // Shan-Chen only
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  const double* ga = dJ_drho_a;
  const double* gb = dJ_drho_b;
  void* tmp = nullptr;
  if (!on_device && (ga != nullptr || gb != nullptr)) {
    if (hipMalloc(&tmp, sizeof(double) * 2 * N) != hipSuccess) {
      (void)hipGetLastError();
      return LB_ENOMEM;
    }
    double* t = static_cast<double*>(tmp);
    bool ok = true;
    if (ga) ok = ok && hipMemcpyAsync(t, ga, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
    if (gb) ok = ok && hipMemcpyAsync(t + N, gb, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      (void)hipFree(tmp);
      return LB_EDEVICE;
    }
    ga = ga ? t : nullptr;
    gb = gb ? t + N : nullptr;
  }
  lb_status st = by_storage(ctx, [&](auto tag) { return adjoint_begin_impl<decltype(tag)::value>(ctx, ga, gb); });
  if (hipStreamSynchronize(ctx->stream) != hipSuccess && st == LB_OK) st = LB_EDEVICE;
  if (tmp) (void)hipFree(tmp);
  return st;
}

lb_status lb_adjoint_step(lb_ctx* ctx, const void* state) {
  if (ctx == nullptr || state == nullptr) return LB_EINVAL;
  if (ctx->model != LB_MODEL_SHAN_CHEN) return LB_EINVAL;  // Shan-Chen only
  if (!ctx->adj_ready) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  return by_storage(ctx, [&](auto tag) { return adjoint_step_impl<decltype(tag)::value>(ctx, state); });
}

lb_status lb_adjoint_result(lb_ctx* ctx, double* dJ_drho_a0, double* dJ_drho_b0, double* dJ_dG, int on_device) {
  if (ctx == nullptr) return LB_EINVAL;
  if (!ctx->adj_ready) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  lb_status st = LB_OK;
  if (dJ_drho_a0 != nullptr || dJ_drho_b0 != nullptr) {
    if (on_device) {
      st = by_storage(ctx, [&](auto tag) { return adjoint_result_impl<decltype(tag)::value>(ctx, dJ_drho_a0, dJ_drho_b0); });
    } else {
      void* tmp = nullptr;
      if (hipMalloc(&tmp, sizeof(double) * 2 * N) != hipSuccess) {
        (void)hipGetLastError();
        return LB_ENOMEM;
      }
      double* t = static_cast<double*>(tmp);
      st = by_storage(ctx, [&](auto tag) { return adjoint_result_impl<decltype(tag)::value>(ctx, t, t + N); });
      bool ok = st == LB_OK;
      if (ok && dJ_drho_a0)
        ok = hipMemcpyAsync(dJ_drho_a0, t, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
      if (ok && dJ_drho_b0)
        ok = hipMemcpyAsync(dJ_drho_b0, t + N, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
      if (ok) ok = hipStreamSynchronize(ctx->stream) == hipSuccess;
      (void)hipGetLastError();
      (void)hipFree(tmp);
      if (st == LB_OK && !ok) st = LB_EDEVICE;
    }
    if (st != LB_OK) return st;
  }
  if (dJ_dG != nullptr) {
    double v = 0.0;
    k_adj_fold<<<1, kBlock, 0, ctx->stream>>>(ctx->adj_partial, blocks_for(ctx->g.N), ctx->adj_dG);
    LB_HIP(hipGetLastError());
    LB_HIP(hipMemcpyAsync(&v, ctx->adj_dG, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    LB_HIP(hipStreamSynchronize(ctx->stream));
    *dJ_dG = v;
  }
  LB_HIP(hipStreamSynchronize(ctx->stream));
  return LB_OK;
}

lb_status lb_adjoint_lambda(lb_ctx* ctx, double* lam, int on_device) {
  if (ctx == nullptr || lam == nullptr) return LB_EINVAL;
  if (!ctx->adj_ready) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t n = static_cast<size_t>(2 * Q) * static_cast<size_t>(ctx->g.N);
  if (on_device) {
    lb_status st = by_storage(ctx, [&](auto tag) { return adjoint_export_impl<decltype(tag)::value>(ctx, lam); });
    if (st != LB_OK) return st;
    LB_HIP(hipStreamSynchronize(ctx->stream));
    return LB_OK;
  }
  void* tmp = nullptr;
  if (hipMalloc(&tmp, sizeof(double) * n) != hipSuccess) {
    (void)hipGetLastError();
    return LB_ENOMEM;
  }
  lb_status st = by_storage(ctx, [&](auto tag) { return adjoint_export_impl<decltype(tag)::value>(ctx, static_cast<double*>(tmp)); });
  bool ok = st == LB_OK && hipMemcpyAsync(lam, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess &&
            hipStreamSynchronize(ctx->stream) == hipSuccess;
  (void)hipGetLastError();
  (void)hipFree(tmp);
  if (st != LB_OK) return st;
  return ok ? LB_OK : LB_EDEVICE;
}

lb_status lb_timing(lb_ctx* ctx, int enable) {
  if (ctx == nullptr) return LB_EINVAL;
  DeviceGuard dg(ctx->p.device);
  if (enable) {
    lb_status st = fold_timing(ctx);
    if (st != LB_OK) return st;
    for (int s = 0; s < SLOT_COUNT; ++s) {
      ctx->t_ms[s] = 0.0;
      ctx->t_n[s] = 0;
    }
  }
  ctx->timing = enable != 0;
  return LB_OK;
}

lb_status lb_timing_read(lb_ctx* ctx, int32_t slot, double* total_ms, int64_t* launches) {
  if (ctx == nullptr || slot < 0 || slot >= SLOT_COUNT) return LB_EINVAL;
  DeviceGuard dg(ctx->p.device);
  lb_status st = fold_timing(ctx);
  if (st != LB_OK) return st;
  if (total_ms != nullptr) *total_ms = ctx->t_ms[slot];
  if (launches != nullptr) *launches = ctx->t_n[slot];
  return LB_OK;
}

// ---- single-fluid step -----------------------------------------------------
lb_status lb1_create(const lb_params* params, lb1_ctx** out) {
  if (out == nullptr) return LB_EINVAL;
  *out = nullptr;
  if (params == nullptr) return LB_EINVAL;
  const lb_params& p = *params;
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return LB_EINVAL;
  if (!is_finite(p.tau[0]) || !(p.tau[0] > 0.5) || !is_finite(p.rho0[0])) return LB_EINVAL;
  if (p.storage != LB_F64 && p.storage != LB_F32 && p.storage != LB_F16_SHIFTED) return LB_EINVAL;
  const long long N = static_cast<long long>(p.nx) * p.ny * p.nz;
  if (N > 0x7fffffffLL - 4096) return LB_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) {
    (void)hipGetLastError();
    return LB_EDEVICE;
  }
  if (p.device < 0 || p.device >= ndev) return LB_EDEVICE;
  DeviceGuard dg(p.device);
  if (!dg.ok) return LB_EDEVICE;
  lb1_ctx* ctx = new (std::nothrow) lb1_ctx();
  if (ctx == nullptr) return LB_ENOMEM;
  ctx->p = p;
  ctx->stream = static_cast<hipStream_t>(p.stream);
  ctx->g.nx = p.nx;
  ctx->g.ny = p.ny;
  ctx->g.nz = p.nz;
  ctx->g.N = static_cast<int>(N);
  ctx->g.Npad = (N + 127) / 128 * 128;
  ctx->elem = p.storage == LB_F64 ? 8 : (p.storage == LB_F32 ? 4 : 2);
  ctx->grid_bytes = ctx->elem * static_cast<size_t>(Q) * static_cast<size_t>(ctx->g.Npad);
  StepCoeffs& c = ctx->c;
  c.om[0] = c.om[1] = 1.0 / p.tau[0];
  c.omc[0] = c.omc[1] = 1.0 - c.om[0];
  c.omf[0] = c.omf[1] = static_cast<float>(c.om[0]);
  c.omcf[0] = c.omcf[1] = static_cast<float>(c.omc[0]);
  for (int i = 0; i < Q; ++i)
    c.shift[0][i] = p.storage == LB_F16_SHIFTED ? static_cast<float>(weight<double>(i) * p.rho0[0]) : 0.0f;
  lb_status st = LB_OK;
  for (int b = 0; b < 2 && st == LB_OK; ++b) st = alloc1(&ctx->grid[b], ctx->grid_bytes);
  if (st == LB_OK) st = alloc1(reinterpret_cast<void**>(&ctx->partial), sizeof(double) * 8 * kTotalsMaxBlocks);
  if (st == LB_OK) st = alloc1(reinterpret_cast<void**>(&ctx->result), sizeof(double) * 8);
  if (st == LB_OK) st = alloc1(reinterpret_cast<void**>(&ctx->flag), sizeof(int) * 4);
  if (st != LB_OK) {
    free1(ctx);
    delete ctx;
    return st;
  }
  *out = ctx;
  return LB_OK;
}

lb_status lb1_destroy(lb1_ctx* ctx) {
  if (ctx == nullptr) return LB_OK;
  DeviceGuard dg(ctx->p.device);
  free1(ctx);
  delete ctx;
  return LB_OK;
}

lb_status lb1_set_stream(lb1_ctx* ctx, void* stream) {
  if (ctx == nullptr) return LB_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  ctx->p.stream = stream;
  return LB_OK;
}

lb_status lb1_set_fields(lb1_ctx* ctx, const double* rho, const double* u, const uint8_t* solid, int on_device) {
  if (ctx == nullptr || rho == nullptr) return LB_EINVAL;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  const double* dr = rho;
  const double* du = u;
  void* tmp = nullptr;
  if (!on_device) {
    if (hipMalloc(&tmp, sizeof(double) * (u != nullptr ? 4 : 1) * N) != hipSuccess) {
      (void)hipGetLastError();
      return LB_ENOMEM;
    }
    double* t = static_cast<double*>(tmp);
    bool ok = hipMemcpyAsync(t, rho, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
    if (ok && u != nullptr)
      ok = hipMemcpyAsync(t + N, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      (void)hipFree(tmp);
      return LB_EDEVICE;
    }
    dr = t;
    du = u != nullptr ? t + N : nullptr;
  }
  auto finish = [&](lb_status st) {
    if (tmp != nullptr) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(tmp);
    }
    return st;
  };
  int bad = 0;
  if (hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream) != hipSuccess) return finish(LB_EDEVICE);
  k_validate_fields<<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(dr, dr, du, ctx->g.N, ctx->flag, 0);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&bad, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return finish(LB_EDEVICE);
  if (bad) return finish(LB_EINVAL);
  if (solid != nullptr) {
    if (ctx->mask == nullptr && alloc1(reinterpret_cast<void**>(&ctx->mask), N) != LB_OK) return finish(LB_ENOMEM);
    if (hipMemcpyAsync(ctx->mask, solid, N, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       ctx->stream) != hipSuccess) {
      (void)hipGetLastError();
      return finish(LB_EDEVICE);
    }
  }
  ctx->has_solid = solid != nullptr;
  ctx->np = 0;  // new fields drop the particles
  // solid nodes are never written by a step, so both grids start from zero
  for (int b = 0; b < 2; ++b)
    if (hipMemsetAsync(ctx->grid[b], 0, ctx->grid_bytes, ctx->stream) != hipSuccess) return finish(LB_EDEVICE);
  ctx->cur = 0;
  const uint8_t* m = ctx->has_solid ? ctx->mask : nullptr;
  lb_status st = by_storage_id(ctx->p.storage, [&](auto tag) {
    constexpr int ST = decltype(tag)::value;
    k1_init<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
        dr, du, m, static_cast<typename StorageTraits<ST>::store_t*>(ctx->grid[0]), ctx->g, ctx->c);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_EDEVICE;
  });
  if (st == LB_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = LB_EDEVICE;
  if (st == LB_OK) ctx->has_state = true;
  return finish(st);
}

lb_status lb1_step(lb1_ctx* ctx, int32_t n) {
  if (ctx == nullptr || n < 0) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  if (n == 0) return LB_OK;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  if (ctx->np > 0) {
    // fluid step, forces and leap-frog, owner map of the new positions, covering/uncovering
    return by_storage_id(ctx->p.storage, [&](auto tag) {
      constexpr int ST = decltype(tag)::value;
      using store = typename StorageTraits<ST>::store_t;
      if constexpr (ST == ST_F16S) {
        return LB_EINVAL;
      } else {
        for (int s = 0; s < n; ++s) {
          const store* fin = static_cast<const store*>(ctx->grid[ctx->cur]);
          store* fout = static_cast<store*>(ctx->grid[ctx->cur ^ 1]);
          const int* own = ctx->owner[ctx->ocur];
          int* own_new = ctx->owner[ctx->ocur ^ 1];
          k1p_step<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(fin, fout, own, ctx->rho_buf, ctx->g,
                                                                         ctx->c);
          kp_force_move<ST><<<ctx->np, kPartThreads, 0, ctx->stream>>>(fout, own, ctx->rho_buf, ctx->ps, ctx->g,
                                                                       ctx->c);
          kp_owner_fill<<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(own_new, ctx->g.N);
          kp_owner_scatter<<<ctx->np, kBlock, 0, ctx->stream>>>(own_new, ctx->ps, ctx->g);
          kp_remap<ST><<<ctx->np, kPartThreads, 0, ctx->stream>>>(fout, own, own_new, ctx->mask, ctx->ps, ctx->g,
                                                                  ctx->c);
          LB_HIP(hipGetLastError());
          ctx->cur ^= 1;
          ctx->ocur ^= 1;
        }
        return LB_OK;
      }
    });
  }
  const uint8_t* m = ctx->has_solid ? ctx->mask : nullptr;
  return by_storage_id(ctx->p.storage, [&](auto tag) {
    constexpr int ST = decltype(tag)::value;
    using store = typename StorageTraits<ST>::store_t;
    for (int s = 0; s < n; ++s) {
      const store* fin = static_cast<const store*>(ctx->grid[ctx->cur]);
      store* fout = static_cast<store*>(ctx->grid[ctx->cur ^ 1]);
      if (m) k1_step<ST, true><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(fin, fout, m, ctx->g, ctx->c);
      else k1_step<ST, false><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(fin, fout, m, ctx->g, ctx->c);
      LB_HIP(hipGetLastError());
      ctx->cur ^= 1;
    }
    return LB_OK;
  });
}

lb_status lb1_moments(lb1_ctx* ctx, double* rho, double* u, int on_device) {
  if (ctx == nullptr) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  double* dr = rho;
  double* du = u;
  void* tmp = nullptr;
  if (!on_device) {
    if (hipMalloc(&tmp, sizeof(double) * 4 * N) != hipSuccess) {
      (void)hipGetLastError();
      return LB_ENOMEM;
    }
    dr = rho ? static_cast<double*>(tmp) : nullptr;
    du = u ? static_cast<double*>(tmp) + N : nullptr;
  }
  const uint8_t* m = solid_of(ctx);
  lb_status st = by_storage_id(ctx->p.storage, [&](auto tag) {
    constexpr int ST = decltype(tag)::value;
    k1_moments<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
        static_cast<const typename StorageTraits<ST>::store_t*>(ctx->grid[ctx->cur]), m, dr, du, ctx->g, ctx->c);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_EDEVICE;
  });
  bool ok = st == LB_OK;
  if (ok && !on_device && rho)
    ok = hipMemcpyAsync(rho, dr, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
  if (ok && !on_device && u)
    ok = hipMemcpyAsync(u, du, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(ctx->stream) == hipSuccess;
  (void)hipGetLastError();
  if (tmp != nullptr) (void)hipFree(tmp);
  if (st != LB_OK) return st;
  return ok ? LB_OK : LB_EDEVICE;
}

lb_status lb1_get_populations(lb1_ctx* ctx, double* f, int on_device) {
  if (ctx == nullptr || f == nullptr) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const size_t N = static_cast<size_t>(ctx->g.N);
  if (!on_device && ctx->plane == nullptr) {
    lb_status st = alloc1(reinterpret_cast<void**>(&ctx->plane), sizeof(double) * N);
    if (st != LB_OK) return st;
  }
  const uint8_t* m = solid_of(ctx);
  for (int plane = 0; plane < Q; ++plane) {
    double* dst = on_device ? f + plane * N : ctx->plane;
    lb_status st = by_storage_id(ctx->p.storage, [&](auto tag) {
      constexpr int ST = decltype(tag)::value;
      k_decode_plane<ST><<<blocks_for(ctx->g.N), kBlock, 0, ctx->stream>>>(
          static_cast<const typename StorageTraits<ST>::store_t*>(ctx->grid[ctx->cur]), dst, m, plane, ctx->g, ctx->c);
      return hipGetLastError() == hipSuccess ? LB_OK : LB_EDEVICE;
    });
    if (st != LB_OK) return st;
    if (!on_device) {
      LB_HIP(hipMemcpyAsync(f + plane * N, ctx->plane, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
      LB_HIP(hipStreamSynchronize(ctx->stream));
    }
  }
  LB_HIP(hipStreamSynchronize(ctx->stream));
  return LB_OK;
}

lb_status lb1_totals(lb1_ctx* ctx, double out[4], int* nonfinite) {
  if (ctx == nullptr || out == nullptr) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  int blocks = blocks_for(ctx->g.N);
  if (blocks > kTotalsMaxBlocks) blocks = kTotalsMaxBlocks;
  const uint8_t* m = solid_of(ctx);
  lb_status st = by_storage_id(ctx->p.storage, [&](auto tag) {
    constexpr int ST = decltype(tag)::value;
    k_totals_partial<ST, 1><<<blocks, kBlock, 0, ctx->stream>>>(
        static_cast<const typename StorageTraits<ST>::store_t*>(ctx->grid[ctx->cur]), m, ctx->g, ctx->c, ctx->partial);
    k_totals_final<<<1, kBlock, 0, ctx->stream>>>(ctx->partial, blocks, ctx->result);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_EDEVICE;
  });
  if (st != LB_OK) return st;
  double r[8] = {0};
  LB_HIP(hipMemcpyAsync(r, ctx->result, sizeof(double) * kTotals, hipMemcpyDeviceToHost, ctx->stream));
  LB_HIP(hipStreamSynchronize(ctx->stream));
  out[0] = r[0];
  out[1] = r[2];
  out[2] = r[3];
  out[3] = r[4];
  const int nf = r[5] != 0.0 ? 1 : 0;
  if (nonfinite != nullptr) *nonfinite = nf;
  return nf ? LB_ENONFINITE : LB_OK;
}

lb_status lb1_set_particles(lb1_ctx* ctx, int32_t count, double radius, double mass, const double* pos,
                            const double* vel, const double* omega) {
  if (ctx == nullptr || count < 0) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  if (count > 0 && (pos == nullptr || ctx->has_solid || ctx->p.storage == LB_F16_SHIFTED)) return LB_EINVAL;
  return set_particles_common<1>(ctx, count, radius, mass, pos, vel, omega,
                                 [](void** ptr, size_t bytes) { return alloc1(ptr, bytes); });
}

lb_status lb1_get_particles(lb1_ctx* ctx, double* pos, double* vel, double* omega, double* force, double* torque) {
  if (ctx == nullptr) return LB_EINVAL;
  return get_particles_common(ctx, pos, vel, omega, force, torque);
}

lb_status lb_set_particles(lb_ctx* ctx, int32_t count, double radius, double mass, const double* pos,
                           const double* vel, const double* omega) {
  if (ctx == nullptr || count < 0) return LB_EINVAL;
  if (!ctx->has_state) return LB_ESTATE;
  if (count > 0 && (pos == nullptr || ctx->model != LB_MODEL_COLOUR_GRADIENT || ctx->has_solid ||
                    ctx->p.storage == LB_F16_SHIFTED))
    return LB_EINVAL;
  DeviceGuard dg(ctx->p.device);
  if (!dg.ok) return LB_EDEVICE;
  const lb_status st = set_layout(ctx, false);  // placing and releasing particles address the structure of arrays
  if (st != LB_OK) return st;
  return set_particles_common<2>(ctx, count, radius, mass, pos, vel, omega,
                                 [ctx](void** ptr, size_t bytes) { return dev_alloc(ctx, ptr, bytes); });
}

lb_status lb_get_particles(lb_ctx* ctx, double* pos, double* vel, double* omega, double* force, double* torque) {
  if (ctx == nullptr) return LB_EINVAL;
  return get_particles_common(ctx, pos, vel, omega, force, torque);
}

}  // extern "C"

// mg_engine.hip -- host-side engine and C ABI of the multigrid solver (see include/mg355.h).
//
// A context owns one pooled device workspace (grown on demand, reused across solves) holding
// the level hierarchy, the per-level boundary face arrays and the reduction scratch.  A solve
// enqueues everything on the caller's stream; the host reads one scalar per cycle for the
// stopping test of Sec. 2.3.7.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "mg355.h"
#include "mg_blocks.h"
#include "mg_fused.h"
#include "mg_launch.h"
#include "mg_march.h"
#include "mg_tile.h"
#include "mg_tblock.h"

using namespace mg;

// ---- static device scratch of the allocation-free solve (mg_solve_noalloc)
//
// One array per device for the life of the process.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is used.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Device address of `scratch` on `device` (the caller has made it current); looked up once.
char* static_scratch(int device, hipError_t* err) {
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* ptr = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = g_scratch_err[device] == hipSuccess ? static_cast<char*>(ptr) : nullptr;
    g_scratch_done[device] = true;
  }
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}
}  // namespace

struct mg_ctx {
  int device = 0;
  std::string err;
  // device address of the static scratch on this context's device (allocation-free solve)
  char* static_scratch = nullptr;
  hipError_t static_scratch_err = hipSuccess;
  // device bytes this context may hold (workspace, operator scratch, reduction scratch);
  // 0 = no limit
  size_t hbm_budget = 0;
  size_t lds_per_block = 65536;
  int tail64_top = 3;          // highest FP64 level held by the LDS coarse tail
  bool tail_fas = false;       // the tail also runs FAS cycles (LDS for phibar beside u and f)
  char* ws = nullptr;
  size_t ws_cap = 0;
  double* part = nullptr;      // reduction partials
  double* scal = nullptr;      // device scalars: [0] sum rho, [1] sum f^2, [2] defect^2, [3] sum phi,
                               // [8..13] sum b^2 per face, [16..47] multipole scratch
  double* hscal = nullptr;     // pinned host mirror of scal
  // the stopping test's squared norm as the device publishes it after each cycle (coherent
  // pinned memory: [0] the value's bits, [1] the publishing launch's sequence number); pub_ok
  // turns false if a publication ever fails to arrive (blocking copies from then on)
  unsigned long long* hpub = nullptr;
  unsigned long long pub_seq = 0;
  bool pub_ok = true;
  // timing of the last solve
  hipEvent_t ev0 = nullptr, ev_setup = nullptr, ev_fmg = nullptr;
  std::vector<hipEvent_t> ev_cycle;
  double setup_ms = 0, fmg_ms = 0;
  std::vector<double> cycle_ms;
  // kernel timing of the finest-level smoothing kernels: an event pair per launch (from the
  // kernel's own dispatch, or recorded around a split pass), then per kernel name the launch
  // count, summed duration and algorithmic bytes per launch
  int ktiming = 0;
  std::vector<hipEvent_t> kev;
  std::vector<int> kev_id;
  struct KStat {
    std::string name;
    int launches = 0;
    double ms = 0, bytes = 0;
  };
  std::vector<KStat> kstats;
  // scratch of the operator entry points (ping-pong partner of a caller's array)
  void* op_scratch = nullptr;
  size_t op_scratch_cap = 0;
  // second stream and events for the split passes of levels with x or y walls, and whether the
  // solver uses them ("split" setting: -1 = default (on), 0 = off, 1 = on)
  MarchAux aux;
  int split = -1;
  // mixed precision: FP32 V-cycles per outer defect-correction step ("inner" setting; -1 =
  // chosen per step by the solver), and how many the last solve ran
  int inner = -1;
  int last_inner = 0;
  // workspace of the refined-mesh solve (grown on demand, kept across calls)
  double* amr_ws = nullptr;
  size_t amr_ws_cap = 0;
  // block-sweep schedules chosen by mg_autotune (or set), keyed by (precision, Lm, Lb)
  std::map<int, BlkTune> blk_tune;
  // MeshBlock layout: sweep the block levels of at least fused_min_n cells per side with the
  // streaming z-marching passes (1) or with the per-block halo-tile sweeps (0); -1 = default
  int blk_zmarch[2] = {-1, -1};
  // dense fused passes: whether the restricted defect (bit 0) and the finest-level norm
  // (bit 1) run fused into the last smoothing pass or as separate defect-only passes,
  // keyed by (precision, level); absent = the default of split_default()
  std::map<int, int> pass_split;
  // smallest level swept by the fused z-marching passes (smaller levels: one launch per
  // operator) and highest level of the LDS coarse tail, per precision [0 = FP64, 1 = FP32];
  // 0 = the built-in default
  int fused_min_n[2] = {0, 0};
  int tail_top[2] = {0, 0};
  // large-level smoothing: 1 = temporally blocked passes (two sweeps per pass over HBM),
  // 0 = one sweep per pass; -1 = the built-in default
  int tblock[2] = {-1, -1};
  // V(2,2) legs as two-sweep streaming passes (down: two sweeps + restricted defect; up:
  // prolongation + two sweeps [+ norm]): 0 = off, 1 = on levels whose faces are all periodic,
  // 2 = on every level; -1 = the built-in default (2)
  int march[2] = {-1, -1};
  // V(2,2) legs of the levels 32^3 .. 128^3 (and the MeshBlock levels below the streaming
  // passes) as one region-tile launch each: 1 = on (default), 0 = per-operator launches
  int tile[2] = {-1, -1};
};

// refined-mesh solve (mg_amr.hip); part: device partials (kMaxPartials x 32 doubles), hpart:
// host partials (kMaxPartials x (MG_AMR_MAX_LEVELS + 1) doubles); *pool / *pool_cap: the
// caller's workspace, grown (up to `room` bytes) when the mesh needs more
int amr_solve_impl(int device, const mg_params* p, const mg_amr_mesh* m, const mg_bc* bc, const double* const* rho,
                   double* const* phi, double* hist, int* n_hist, void* stream, double* part, double* hpart,
                   double** pool, size_t* pool_cap, size_t room, std::string* err);

namespace {

constexpr int kScal = 64;
constexpr int kMpoleOff = 16;

int fail(mg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_CHECK(ctx, call)                                                                     \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail((ctx), MG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

bool is_pow2(long long n) { return n >= 1 && (n & (n - 1)) == 0; }

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t cells(int l) { return (size_t)1 << (3 * l); }
size_t face_sz(int l) { return (size_t)((1 << l) + 2) * (size_t)((1 << l) + 2); }

// Layout of the workspace for one (n, precision).
struct Layout {
  int L = 0;
  bool mixed = false;
  size_t f64L = 0;             // FP64 finest source
  size_t u64[16], f64[16];     // FP64 levels 0..L-1 (FP64 mode)
  size_t u32[16], f32[16];     // FP32 levels 0..L (mixed mode)
  size_t u2[16];               // second (ping-pong) buffer of the levels swept by fused passes
  size_t phi2 = (size_t)-1;    // mixed mode: ping-pong partner of the caller's FP64 phi
  size_t faces[16];            // 6 extended face arrays per level
  size_t pbar[16];             // FAS: restricted potential of levels 0..L-1
  size_t total = 0;
};

// Lb >= 0: MeshBlock layout with 2^Lb blocks per side (levels above Lb are block levels,
// each swept out of place, so each has a ping-pong partner).
// fas: the restricted-potential arrays of the Full Approximation Scheme (FP64 levels below L).
Layout make_layout(int n, int precision, int Lb = -1, bool fas = false) {
  Layout y;
  y.L = ilog2(n);
  y.mixed = precision == MG_PREC_MIXED;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  y.f64L = take(cells(y.L) * 8);
  if (y.mixed && n >= kFusedMinN) y.phi2 = take(cells(y.L) * 8);
  for (int l = 0; l <= y.L; ++l) {
    y.u64[l] = y.f64[l] = y.u32[l] = y.f32[l] = 0;
    if (!y.mixed && l < y.L) {
      y.u64[l] = take(cells(l) * 8);
      y.f64[l] = take(cells(l) * 8);
    }
    if (y.mixed) {
      y.u32[l] = take(cells(l) * 4);
      y.f32[l] = take(cells(l) * 4);
    }
    y.faces[l] = take(6 * face_sz(l) * 8);
    y.pbar[l] = (fas && l < y.L) ? take(cells(l) * 8) : (size_t)-1;
    y.u2[l] = (size_t)-1;
    if ((1 << l) >= kTileMinN || (Lb >= 0 && l > Lb)) y.u2[l] = take(cells(l) * (y.mixed ? 4 : 8));
  }
  y.total = off;
  return y;
}

// log2 of the blocks per side of a MeshBlock-layout solve, -1 for the dense layout.
int layout_lb(const mg_params* p) {
  if (p->layout != MG_LAYOUT_BLOCKS || !is_pow2(p->block_n) || p->block_n < 2 || p->block_n >= p->n) return -1;
  return ilog2(p->n / p->block_n);
}

int validate(mg_ctx* c, const mg_params* p, const mg_bc* bc) {
  if (!p || !bc) return fail(c, MG_ERR_INVALID_ARG, "null params or bc");
  if (!is_pow2(p->n) || p->n < 2 || p->n > 2048) return fail(c, MG_ERR_INVALID_ARG, "n must be a power of two in [2, 2048]");
  if (!(p->dx > 0) || !std::isfinite(p->dx)) return fail(c, MG_ERR_INVALID_ARG, "dx must be positive");
  if (p->npre < 0 || p->npre > 4 || p->npost < 0 || p->npost > 4) return fail(c, MG_ERR_INVALID_ARG, "npre/npost in 0..4");
  if (!(p->omega > 0 && p->omega < 2)) return fail(c, MG_ERR_INVALID_ARG, "omega in (0, 2)");
  if (p->max_cycles < 0 || p->max_cycles > 1000 || p->fixed_cycles < 0 || p->fixed_cycles > 1000)
    return fail(c, MG_ERR_INVALID_ARG, "cycle counts in 0..1000");
  if (p->mode != MG_MODE_FMG && p->mode != MG_MODE_MGI) return fail(c, MG_ERR_INVALID_ARG, "bad mode");
  if (p->precision != MG_PREC_FP64 && p->precision != MG_PREC_MIXED) return fail(c, MG_ERR_INVALID_ARG, "bad precision");
  if (p->layout != MG_LAYOUT_DENSE && p->layout != MG_LAYOUT_BLOCKS) return fail(c, MG_ERR_INVALID_ARG, "bad layout");
  if (p->layout == MG_LAYOUT_BLOCKS &&
      (!is_pow2(p->block_n) || p->block_n < 2 || p->block_n > (1 << kBlkMaxLm) || p->block_n >= p->n ||
       p->n / p->block_n > 1024))
    return fail(c, MG_ERR_INVALID_ARG, "block_n must be a power of two in [2, 16], below n, with at most 1024 blocks per side");
  for (int f = 0; f < 6; ++f)
    if (bc->kind[f] < MG_BC_PERIODIC || bc->kind[f] > MG_BC_MULTIPOLE) return fail(c, MG_ERR_INVALID_ARG, "bad face kind");
  for (int a = 0; a < 3; ++a)
    if ((bc->kind[2 * a] == MG_BC_PERIODIC) != (bc->kind[2 * a + 1] == MG_BC_PERIODIC))
      return fail(c, MG_ERR_INVALID_ARG, "periodic faces must be paired per axis");
  if (bc->lmax < 0 || bc->lmax > 4) return fail(c, MG_ERR_INVALID_ARG, "lmax in 0..4");
  if (p->scheme != MG_SCHEME_CS && p->scheme != MG_SCHEME_FAS) return fail(c, MG_ERR_INVALID_ARG, "bad scheme");
  if (p->scheme == MG_SCHEME_FAS && (p->precision != MG_PREC_FP64 || p->layout != MG_LAYOUT_DENSE))
    return fail(c, MG_ERR_UNSUPPORTED, "FAS runs in FP64 on the dense layout");
  return MG_OK;
}

LevelBC to_level_bc(const mg_level_bc* b) {
  LevelBC r;
  for (int f = 0; f < 6; ++f) {
    r.kind[f] = b ? (b->kind[f] == MG_BC_MULTIPOLE ? MG_BC_FIXED : b->kind[f]) : MG_BC_PERIODIC;
    r.b[f] = b ? b->b[f] : nullptr;
  }
  return r;
}

// Device bytes the context holds besides its workspace and operator scratch.
constexpr size_t kFixedBytes = sizeof(double) * (kMaxPartials * 32 + kScal);

// Would holding `bytes` more (beyond what the context holds now, less `freed`) exceed its budget?
bool over_budget(const mg_ctx* c, size_t bytes, size_t freed) {
  if (c->hbm_budget == 0) return false;
  const size_t held = kFixedBytes + c->ws_cap + c->op_scratch_cap + c->amr_ws_cap - freed;
  return held + bytes > c->hbm_budget;
}

int ensure_ws(mg_ctx* c, size_t bytes) {
  if (bytes <= c->ws_cap) return MG_OK;
  if (over_budget(c, bytes, c->ws_cap))
    return fail(c, MG_ERR_OOM, "workspace of " + std::to_string(bytes) + " bytes exceeds the context's HBM budget of " +
                                   std::to_string(c->hbm_budget) + " bytes");
  if (c->ws) {
    HIP_CHECK(c, hipDeviceSynchronize());
    HIP_CHECK(c, hipFree(c->ws));
    c->ws = nullptr;
    c->ws_cap = 0;
  }
  hipError_t e = hipMalloc((void**)&c->ws, bytes);
  if (e != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return fail(c, MG_ERR_OOM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
  }
  c->ws_cap = bytes;
  return MG_OK;
}

// Per-solve plan: typed level pointers and boundary descriptions.
template <typename T>
struct Hier {
  int L = 0, T_top = 0;
  T* u[16];
  T* u2[16];          // ping-pong partner of u[l] for fused levels, else nullptr
  T* f[16];
  double h[16];
  LevelBC phys[16];
  LevelBC hom;
  int npre = 2, npost = 2;
  double omega = 1.15;
};

// Smallest level side on which the two-sweep passes run: kMarchMinN, or the one-sweep passes'
// threshold ("fusedmin") when that was set larger.
template <typename T>
int march_min_n(const mg_ctx* c) {
  const int v = c->fused_min_n[sizeof(T) == 8 ? 0 : 1];
  return v > 0 ? std::max(kMarchMinN, v) : kMarchMinN;
}

// Does a MeshBlock level of 2^l cells per side fit the two-sweep passes' 32-bit block index?
inline bool blk_march_fits(int l) { return 3 * l < 32; }

struct Solver {
  mg_ctx* c;
  hipStream_t s;
  bool use_fused = true;
  // device reduction scratch of this solve (partials, scalars) and kernel timing on/off
  double* part = nullptr;
  double* scal = nullptr;
  int ktiming = 0;
  int fused_min_n64 = kFusedDefaultMinN, fused_min_n32 = kFusedDefaultMinN;
  // the next top-level V-cycle starts from u = 0 without u having been cleared: its first
  // sweep must not read u (set by the caller, consumed by vcycle)
  bool zero_start = false;
  // the first pre-smoothing sweep of the next top-level V-cycle has already run (the head
  // pass, which also measured the residual of its input): its result is in u2 (consumed by
  // vcycle)
  bool head_done = false;

  // the first leg of the next top-level V-cycle has already been queued (down_ahead): the
  // next top-level vcycle / vcycle_blk skips it
  bool down_done = false;

  // The down leg of dense level l of a V(2,2) cycle in one launch: the two-sweep pass
  // (march) or the region-tile leg.  It reads u and f and writes only u2 and the coarse
  // level's source and correction.  zin: u is zero and not read.
  template <typename T>
  void down_leg(Hier<T>& H, int l, const LevelBC& bc, bool march, bool zin, bool timed) {
    const int n = 1 << l;
    const double cellsT = (double)cells(l) * sizeof(T);
    if (timed) kernel_begin(true);
    if (march) {
      march_down<T>(zin ? nullptr : H.u[l], H.u2[l], H.f[l], H.f[l - 1], H.u[l - 1], n, H.h[l], H.omega, bc, s, 0,
                    aux_of());
      // algorithmic bytes: u and f read, u written, coarse source and correction written
      if (timed) kernel_end(march_name<T>(false, false, bc), 3 * cellsT + cellsT / 4);
    } else {
      tile_down<T>(H.u[l], H.u2[l], H.f[l], H.f[l - 1], H.u[l - 1], n, 0, 0, H.h[l], H.omega, bc, s);
      if (timed) kernel_end(tile_name<T>(false, false), 3 * cellsT + cellsT / 4);
    }
  }
  // The same for MeshBlock level l (big: the two-sweep pass across blocks).
  template <typename T>
  void blk_down_leg(Hier<T>& H, int l, const LevelBC& bc, bool big, bool timed) {
    const int nl = 1 << l, Lm = l - Lb;
    const double cellsT = (double)cells(l) * sizeof(T);
    if (timed) kernel_begin(true);
    if (big) march_down<T>(H.u[l], H.u2[l], H.f[l], H.f[l - 1], H.u[l - 1], nl, H.h[l], H.omega, bc, s, Lm, aux_of());
    else tile_down<T>(H.u[l], H.u2[l], H.f[l], H.f[l - 1], H.u[l - 1], nl, Lm, Lb, H.h[l], H.omega, bc, s);
    if (timed) kernel_end(big ? march_name<T>(false, false, bc, true) : tile_name<T>(false, false, true),
                          3 * cellsT + cellsT / 4);
  }

  // Queues the next top-level V-cycle's first leg now, before the host has read this cycle's
  // norm (the solve loop decides when): FP64 correction-scheme cycles whose finest-level down
  // leg is one of the single launches above, under the same conditions vcycle / vcycle_blk
  // apply.  If the solve stops after all, nothing that leg wrote is read.  Returns whether it
  // queued the leg (then down_done is set).
  bool down_ahead(Hier<double>& H, const LevelBC& bc) {
    const int L = H.L;
    const bool timed = timed_top && ktiming;
    if (H.npre != 2 || H.npost != 2 || L == H.T_top) return false;
    if (Lb < 0) {
      if (march_on<double>(H, L, bc)) down_leg<double>(H, L, bc, true, false, timed);
      else if ((1 << L) < fused_min_n64 && tile_on<double>(H, L)) down_leg<double>(H, L, bc, false, false, timed);
      else return false;
    } else {
      if (L <= Lb) return false;
      const bool big = c->blk_zmarch[0] != 0 && (1 << L) >= march_min<double>() && march_blk_on<double>(H, L, bc);
      if (!big && !tile_on<double>(H, L)) return false;
      blk_down_leg<double>(H, L, bc, big, timed);
    }
    down_done = true;
    return true;
  }
  // The timing record of a leg queued ahead and then not used (the last two events).
  void drop_ahead_timing() {
    if (!(timed_top && ktiming) || c->kev.size() < 2 || c->kev_id.empty()) return;
    for (int q = 0; q < 2; ++q) {
      (void)hipEventDestroy(c->kev.back());
      c->kev.pop_back();
    }
    c->kev_id.pop_back();
  }

  // hook: the launcher that follows takes the launch-timing hook (one kernel timed by its own
  // dispatch, no marker packets around it); otherwise events are recorded around the launcher
  bool hooked = false;
  void kernel_begin(bool hook = false) {
    hipEvent_t e;
    (void)hipEventCreate(&e);
    if (hook) {
      LaunchTiming& t = launch_timing();
      t.e0 = e;
      (void)hipEventCreate(&t.e1);
      t.armed = true;
      hooked = true;
    } else {
      (void)hipEventRecord(e, s);
    }
    c->kev.push_back(e);
  }
  // algorithmic bytes of one launch are recorded with its name
  void kernel_end(const std::string& name, double bytes) {
    hipEvent_t e;
    if (hooked) {
      LaunchTiming& t = launch_timing();
      hooked = false;
      e = t.e1;
      if (t.armed) {   // the launcher did not take the hook: an empty interval here
        t.armed = false;
        (void)hipEventRecord(c->kev.back(), s);
        (void)hipEventRecord(e, s);
      }
    } else {
      (void)hipEventCreate(&e);
      (void)hipEventRecord(e, s);
    }
    c->kev.push_back(e);
    int id = -1;
    for (size_t q = 0; q < c->kstats.size(); ++q)
      if (c->kstats[q].name == name) id = (int)q;
    if (id < 0) {
      c->kstats.push_back(mg_ctx::KStat{name, 0, 0.0, bytes});
      id = (int)c->kstats.size() - 1;
    }
    c->kev_id.push_back(id);
  }

  template <typename T>
  void tail(Hier<T>& H, int mode, const LevelBC& bc_top) {
    TailArgs a;
    std::memset(&a, 0, sizeof(a));
    a.top = H.T_top;
    a.mode = mode;
    a.npre = H.npre;
    a.npost = H.npost;
    a.omega = H.omega;
    for (int l = 0; l <= H.T_top; ++l) {
      a.h[l] = H.h[l];
      a.phys[l] = H.phys[l];
      a.fg[l] = H.f[l];
    }
    a.bc_top = bc_top;
    a.hom = H.hom;
    a.ug = H.u[H.T_top];
    launch_tail<T>(a, s);
  }

  // Fusion schedule of level l's defect stages: bit 0 = restricted defect as its own pass,
  // bit 1 = norm as its own pass.  Default: the restricted defect fused into the last
  // pre-sweep; the norm fused into the last post-sweep in FP32 and its own pass in FP64 (the
  // fused FP64 sweep + norm runs short of registers).
  template <typename T>
  int split_of(int l) const {
    auto it = c->pass_split.find((sizeof(T) == 8 ? 0 : 1000) + l);
    if (it != c->pass_split.end()) return it->second;
    return sizeof(T) == 8 ? 2 : 0;
  }

  // Does level l run its V(2,2) legs as the two-sweep streaming passes (down: two sweeps and
  // the restricted defect in one pass; up: prolongation, two sweeps and the norm in one)?
  template <typename T>
  bool march_on(const Hier<T>& H, int l, const LevelBC& bc) const {
    const int mode = c->march[sizeof(T) == 8 ? 0 : 1] < 0 ? 2 : c->march[sizeof(T) == 8 ? 0 : 1];
    if (mode == 0 || !use_fused || !H.u2[l] || l == H.T_top || Lb >= 0 || H.npre != 2 || H.npost != 2) return false;
    if ((1 << l) < march_min<T>() || tblock_on<T>()) return false;
    if (mode == 1)
      for (int f = 0; f < 6; ++f)
        if (bc.kind[f] != BC_PERIODIC) return false;
    return true;
  }

  template <typename T>
  int march_min() const {
    return march_min_n<T>(c);
  }

  // the second stream of the split passes (null: one launch per pass)
  const MarchAux* aux_of() const { return c->split == 0 ? nullptr : &c->aux; }

  // May MeshBlock level l run the two-sweep streaming passes (the "march" setting for its
  // faces)?  Those passes index the block layout in 32 bits, so the level must hold fewer than
  // 2^32 cells (every level up to 1024^3); larger ones take the block streaming sweeps.
  template <typename T>
  bool march_blk_on(const Hier<T>& H, int l, const LevelBC& bc) const {
    const int mode = c->march[sizeof(T) == 8 ? 0 : 1] < 0 ? 2 : c->march[sizeof(T) == 8 ? 0 : 1];
    if (mode == 0 || H.npre != 2 || H.npost != 2 || !blk_march_fits(l)) return false;
    if (mode == 1)
      for (int f = 0; f < 6; ++f)
        if (bc.kind[f] != BC_PERIODIC) return false;
    return true;
  }

  // Does level l (side n) run its V(2,2) legs as region-tile launches (one per leg)?
  template <typename T>
  bool tile_on(const Hier<T>& H, int l) const {
    const int v = c->tile[sizeof(T) == 8 ? 0 : 1];
    const int n = 1 << l;
    return (v < 0 || v == 1) && H.u2[l] && l != H.T_top && H.npre == 2 && H.npost == 2 && n >= kTileMinN &&
           n <= kTileMaxN;
  }

  // FP64, dense: can the first pre-sweep of the finest level's V-cycle run as a head pass (a
  // one-sweep streaming pass that also takes the residual norm of its input)?  Not when the
  // finest level runs the two-sweep passes, whose up pass takes the norm of the cycle's result.
  bool head_possible(const Hier<double>& H) const {
    const int L = H.L;
    return use_fused && H.u2[L] && L != H.T_top && Lb < 0 && (1 << L) >= fused_min_n64 && !tblock_on<double>() &&
           H.npre >= 1 && ((split_of<double>(L) & 1) || H.npre >= 2) && !march_on<double>(H, L, H.phys[L]);
  }

  // The head pass: first pre-sweep of the next V-cycle (u -> u2) and the residual norm of u
  // (the iterate the stopping test of Sec. 2.3.7 is about) into scal[2].
  void head(Hier<double>& H, const LevelBC& bc) {
    const int L = H.L, n = 1 << L;
    const bool timed = timed_top && ktiming;
    if (timed) kernel_begin();
    const int np = fused_sweep_input_norm<double>(H.u[L], H.u2[L], H.f[L], part, n, H.h[L], H.omega, bc, s);
    if (timed) kernel_end(fused_pass_name<double>(false, 3), 3.0 * (double)cells(L) * sizeof(double));
    launch_sum_partials(part, np, scal + 2, s);
    head_done = true;
  }

  template <typename T>
  bool tblock_on() const {
    const int v = c->tblock[sizeof(T) == 8 ? 0 : 1];
    return v < 0 ? false : v == 1;
  }

  // Alg. 1 on level l (l >= T_top).  At the tail level the whole remaining recursion runs in
  // one LDS-resident workgroup.  Large levels run four fused passes (sweep; sweep + restricted
  // defect; prolonged correction + sweep; sweep [+ defect norm]).  Returns true when the sum
  // of squared defects of the result is in scal[2] (want_norm on a fused finest level).
  template <typename T>
  bool vcycle(Hier<T>& H, int l, const LevelBC& bc, bool top_call, bool want_norm) {
    if (top_call && zero_start) {
      // only the one-sweep fused path starts with a plain sweep that can skip reading u;
      // elsewhere u is cleared first
      const bool fused_first = (use_fused && H.u2[l] && l != H.T_top &&
                                (1 << l) >= (sizeof(T) == 8 ? fused_min_n64 : fused_min_n32) && !tblock_on<T>() &&
                                H.npre >= 1 && !(H.npre == 1 && !(split_of<T>(l) & 1))) ||
                               march_on<T>(H, l, bc);
      if (!fused_first) {
        launch_zero(H.u[l], cells(l) * sizeof(T), s);
        zero_start = false;
      }
    }
    if (l == H.T_top) {
      tail(H, top_call ? TAIL_LOAD_U : 0, bc);
      return false;
    }
    const int n = 1 << l;
    const double h = H.h[l];
    const bool timed = top_call && l == H.L && ktiming;
    const double cellsT = (double)cells(l) * sizeof(T);
    if (march_on<T>(H, l, bc)) {
      // V(2,2) in two streaming passes: down (two sweeps, restricted defect, coarse correction
      // cleared), the coarse recursion, up (prolonged correction, two sweeps, and the norm of
      // the result when asked); the result lands back in u[l] after the two ping-pongs
      const bool zin = top_call && zero_start;
      if (top_call && down_done) down_done = false;   // queued ahead of the stopping test
      else down_leg<T>(H, l, bc, true, zin, timed);
      vcycle(H, l - 1, H.hom, false, false);
      double* npart = want_norm && sizeof(T) == 8 ? part : nullptr;
      if (timed) kernel_begin(true);
      const int np = march_up<T>(H.u2[l], H.u[l], H.f[l], H.u[l - 1], H.hom, npart, n, h, H.omega, bc, s, 0, aux_of());
      // algorithmic bytes: u, f and the coarse correction read, u written
      if (timed) kernel_end(march_name<T>(true, npart != nullptr, bc), 3 * cellsT + cellsT / 8);
      if (npart) launch_sum_partials(part, np, scal + 2, s);
      return npart != nullptr;
    }
    if (n < (sizeof(T) == 8 ? fused_min_n64 : fused_min_n32) && tile_on<T>(H, l)) {
      // a small level: each leg in one region-tile launch
      if (top_call && zero_start) {
        launch_zero(H.u[l], cells(l) * sizeof(T), s);
        zero_start = false;
      }
      if (top_call && down_done) down_done = false;   // queued ahead of the stopping test
      else down_leg<T>(H, l, bc, false, false, timed);
      vcycle(H, l - 1, H.hom, false, false);
      double* npart = want_norm && sizeof(T) == 8 ? part : nullptr;
      if (timed) kernel_begin(true);
      const int np = tile_up<T>(H.u2[l], H.u[l], H.f[l], H.u[l - 1], H.hom, npart, n, 0, 0, h, H.omega, bc, s);
      if (timed) kernel_end(tile_name<T>(true, npart != nullptr), 3 * cellsT + cellsT / 8);
      if (npart) launch_sum_partials(part, np, scal + 2, s);
      return npart != nullptr;
    }
    if (use_fused && H.u2[l] && n >= (sizeof(T) == 8 ? fused_min_n64 : fused_min_n32) && tblock_on<T>()) {
      // temporally blocked: sweeps two at a time per pass; the restricted defect and the norm
      // as defect-only passes
      T* cur = H.u[l];
      T* oth = H.u2[l];
      auto sweeps = [&](int count, const T* ec) {
        int left = count;
        while (left > 0) {
          const int ns = left >= 2 ? 2 : 1;
          if (timed) kernel_begin();
          tb_sweeps<T>(cur, oth, H.f[l], ec, H.hom, ns, n, h, H.omega, bc, s);
          if (timed) kernel_end(tb_name<T>(ns, ec != nullptr), 3 * cellsT + (ec ? cellsT / 8 : 0.0));
          std::swap(cur, oth);
          left -= ns;
          ec = nullptr;
        }
      };
      sweeps(H.npre, nullptr);
      if (H.npre == 0) {
        launch_defect_restrict<T>(cur, H.f[l], H.f[l - 1], H.u[l - 1], n, h, bc, s);
      } else {
        if (timed) kernel_begin();
        fused_defect_restrict<T>(cur, H.f[l], H.f[l - 1], H.u[l - 1], n, h, bc, s);
        if (timed) kernel_end(fused_pass_name<T>(false, 1, false), 2 * cellsT + cellsT / 4);
      }
      vcycle(H, l - 1, H.hom, false, false);
      if (H.npost == 0) {
        launch_prolong<T>(H.u[l - 1], cur, n / 2, H.hom, 0, s);
      } else {
        // the prolonged correction enters with the first sweep (one-sweep pass: the coarse
        // taps leave no registers for a second), the remaining sweeps two per pass
        if (timed) kernel_begin();
        fused_prolong_sweep<T>(cur, oth, H.f[l], H.u[l - 1], H.hom, n, h, H.omega, bc, s);
        if (timed) kernel_end(fused_pass_name<T>(true, 0), 3 * cellsT + cellsT / 8);
        std::swap(cur, oth);
        sweeps(H.npost - 1, nullptr);
      }
      bool normed = false;
      if (want_norm && sizeof(T) == 8) {
        if (timed) kernel_begin();
        const int np = fused_defect_norm<T>(cur, H.f[l], part, n, h, bc, s);
        if (timed) kernel_end(fused_pass_name<T>(false, 2, false), 2 * cellsT);
        launch_sum_partials(part, np, scal + 2, s);
        normed = true;
      }
      if (cur != H.u[l]) (void)hipMemcpyAsync(H.u[l], cur, cells(l) * sizeof(T), hipMemcpyDeviceToDevice, s);
      return normed;
    }
    if (use_fused && H.u2[l] && n >= (sizeof(T) == 8 ? fused_min_n64 : fused_min_n32)) {
      const int split = split_of<T>(l);
      const bool sdef = (split & 1) != 0, snorm = (split & 2) != 0;
      T* cur = H.u[l];
      T* oth = H.u2[l];
      int it0 = 0;
      if (top_call && head_done) {
        std::swap(cur, oth);
        it0 = 1;
        head_done = false;
      }
      for (int it = it0; it < H.npre; ++it) {
        const bool fuse = it == H.npre - 1 && !sdef;
        const bool zin = it == 0 && top_call && zero_start && !fuse;
        if (timed) kernel_begin();
        if (fuse) fused_sweep_defect<T>(cur, oth, H.f[l], H.f[l - 1], H.u[l - 1], n, h, H.omega, bc, s);
        else fused_sweep<T>(zin ? nullptr : cur, oth, H.f[l], n, h, H.omega, bc, s);
        if (timed) kernel_end(fused_pass_name<T>(false, fuse ? 1 : 0), 3 * cellsT + (fuse ? cellsT / 4 : 0.0));
        std::swap(cur, oth);
      }
      if (H.npre == 0) {
        launch_defect_restrict<T>(cur, H.f[l], H.f[l - 1], H.u[l - 1], n, h, bc, s);
      } else if (sdef) {
        if (timed) kernel_begin();
        fused_defect_restrict<T>(cur, H.f[l], H.f[l - 1], H.u[l - 1], n, h, bc, s);
        // algorithmic bytes: u and f read, coarse source and correction written
        if (timed) kernel_end(fused_pass_name<T>(false, 1, false), 2 * cellsT + cellsT / 4);
      }
      vcycle(H, l - 1, H.hom, false, false);
      bool normed = false;
      if (H.npost == 0) launch_prolong<T>(H.u[l - 1], cur, n / 2, H.hom, 0, s);
      for (int it = 0; it < H.npost; ++it) {
        const bool last = it == H.npost - 1;
        if (timed) kernel_begin();
        if (it == 0) {
          fused_prolong_sweep<T>(cur, oth, H.f[l], H.u[l - 1], H.hom, n, h, H.omega, bc, s);
          if (timed) kernel_end(fused_pass_name<T>(true, 0), 3 * cellsT + cellsT / 8);
        } else if (last && want_norm && !snorm) {
          const int np = fused_sweep_norm<T>(cur, oth, H.f[l], part, n, h, H.omega, bc, s);
          if (timed) kernel_end(fused_pass_name<T>(false, 2), 3 * cellsT);
          launch_sum_partials(part, np, scal + 2, s);
          normed = true;
        } else {
          fused_sweep<T>(cur, oth, H.f[l], n, h, H.omega, bc, s);
          if (timed) kernel_end(fused_pass_name<T>(false, 0), 3 * cellsT);
        }
        std::swap(cur, oth);
      }
      if (want_norm && !normed && sizeof(T) == 8) {
        if (timed) kernel_begin();
        const int np = fused_defect_norm<T>(cur, H.f[l], part, n, h, bc, s);
        if (timed) kernel_end(fused_pass_name<T>(false, 2, false), 2 * cellsT);
        launch_sum_partials(part, np, scal + 2, s);
        normed = true;
      }
      if (cur != H.u[l]) (void)hipMemcpyAsync(H.u[l], cur, cells(l) * sizeof(T), hipMemcpyDeviceToDevice, s);
      return normed;
    }
    for (int it = 0; it < H.npre; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        if (timed) kernel_begin();
        launch_half_sweep<T>(H.u[l], H.f[l], n, h, H.omega, colour, bc, s);
        // algorithmic bytes: all of u read, f read and u written on one colour
        if (timed) kernel_end("k_half_sweep", 2 * cellsT);
      }
    launch_defect_restrict<T>(H.u[l], H.f[l], H.f[l - 1], H.u[l - 1], n, h, bc, s);
    vcycle(H, l - 1, H.hom, false, false);
    launch_prolong<T>(H.u[l - 1], H.u[l], n / 2, H.hom, 0, s);
    for (int it = 0; it < H.npost; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        if (timed) kernel_begin();
        launch_half_sweep<T>(H.u[l], H.f[l], n, h, H.omega, colour, bc, s);
        if (timed) kernel_end("k_half_sweep", 2 * cellsT);
      }
    return false;
  }

  // ---- Full Approximation Scheme (Alg. 3), FP64 dense: every level keeps its physical
  // boundary description; pbar[l] holds the restricted potential of level l < L.

  // `count` smoothing sweeps of level l starting from `cur` (H.u[l] or, on levels swept by the
  // streaming passes, either ping-pong array); returns the array holding the result.
  double* fas_sweeps(Hier<double>& H, int l, double* cur, int count, const LevelBC& bc) {
    const int n = 1 << l;
    const bool timed = timed_top && l == H.L && ktiming;
    const double cellsT = (double)cells(l) * sizeof(double);
    if (use_fused && H.u2[l] && n >= fused_min_n64) {
      double* oth = cur == H.u[l] ? H.u2[l] : H.u[l];
      for (int it = 0; it < count; ++it) {
        if (timed) kernel_begin();
        fused_sweep<double>(cur, oth, H.f[l], n, H.h[l], H.omega, bc, s);
        if (timed) kernel_end(fused_pass_name<double>(false, 0), 3 * cellsT);
        std::swap(cur, oth);
      }
      return cur;
    }
    for (int it = 0; it < count; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        if (timed) kernel_begin();
        launch_half_sweep<double>(cur, H.f[l], n, H.h[l], H.omega, colour, bc, s);
        if (timed) kernel_end("k_half_sweep", 2 * cellsT);
      }
    return cur;
  }

  static bool fixes_zero(const LevelBC& bc) {
    for (int f = 0; f < 6; ++f)
      if (bc.kind[f] != BC_PERIODIC && bc.kind[f] != BC_ZERO_GRADIENT) return true;
    return false;
  }

  // done: pre-sweeps of the top level already run by the head pass (result in u2).  want_norm
  // (top level): the two-sweep up pass may leave the sum of squared defects of the result in
  // scal[2]; returns whether it did.
  // Can the LDS tail run the FAS cycle from level l: its FAS form allowed, and no level's
  // description (nor the corrections') carrying face values?
  bool fas_tail_ok(const Hier<double>& H, int l) const {
    if (!c->tail_fas) return false;
    auto valueless = [](const LevelBC& q) {
      for (int f = 0; f < 6; ++f)
        if (q.kind[f] != BC_PERIODIC && q.kind[f] != BC_ZERO_GRADIENT && q.b[f]) return false;
      return true;
    };
    if (!valueless(H.hom)) return false;
    for (int q = 0; q <= l; ++q)
      if (!valueless(H.phys[q])) return false;
    return true;
  }

  bool fas_cycle(Hier<double>& H, double* const* pbar, int l, int done = 0, bool want_norm = false) {
    if (l == 0) {
      // the single cell with its physical conditions, from the iterate phibar; when no face
      // fixes the zero point any value solves it and phibar is kept (zero correction)
      if (fixes_zero(H.phys[0])) launch_coarsest<double>(H.u[0], H.f[0], H.h[0], H.phys[0], s);
      return false;
    }
    if (done == 0 && l <= H.T_top && fas_tail_ok(H, l)) {
      // the whole FAS cycle from level l in one LDS-resident workgroup (levels <= 16^3 whose
      // descriptions carry no face values)
      TailArgs a;
      std::memset(&a, 0, sizeof(a));
      a.top = l;
      a.mode = TAIL_FAS | TAIL_LOAD_U;
      a.npre = H.npre;
      a.npost = H.npost;
      a.omega = H.omega;
      for (int q = 0; q <= l; ++q) {
        a.h[q] = H.h[q];
        a.phys[q] = H.phys[q];
        a.fg[q] = H.f[q];
      }
      a.bc_top = H.phys[l];
      a.hom = H.hom;
      a.ug = H.u[l];
      launch_tail<double>(a, s);
      return false;
    }
    const int n = 1 << l;
    const LevelBC& bc = H.phys[l];
    const bool timed = timed_top && l == H.L && ktiming;
    const double cellsT = (double)cells(l) * sizeof(double);
    if (done == 0 && march_on<double>(H, l, bc)) {
      // V(2,2) legs as the two-sweep passes: down (two sweeps, restricted defect, phibar, the
      // coarse level started from it), steps 5-7 on the coarse level, up (the prolonged
      // correction psi - phibar, two sweeps, and the norm of the result when asked)
      if (timed) kernel_begin(true);
      march_down_fas<double>(H.u[l], H.u2[l], H.f[l], H.f[l - 1], pbar[l - 1], H.u[l - 1], n, H.h[l], H.omega, bc, s);
      // algorithmic bytes: u and f read, u written, three coarse arrays written
      if (timed) kernel_end(march_fas_name<double>(bc), 3 * cellsT + 3 * cellsT / 8);
      launch_fas_source(pbar[l - 1], H.f[l - 1], n / 2, H.h[l - 1], H.phys[l - 1], s);       // 5
      fas_cycle(H, pbar, l - 1);                                                             // 6
      launch_fas_correction(H.u[l - 1], pbar[l - 1], cells(l - 1), s);                       // 7
      double* npart = want_norm ? part : nullptr;
      if (timed) kernel_begin(true);
      const int np = march_up<double>(H.u2[l], H.u[l], H.f[l], H.u[l - 1], H.hom, npart, n, H.h[l], H.omega, bc, s, 0,
                                      aux_of());
      if (timed) kernel_end(march_name<double>(true, npart != nullptr, bc), 3 * cellsT + cellsT / 8);
      if (npart) launch_sum_partials(part, np, scal + 2, s);
      return npart != nullptr;
    }
    if (done == 0 && n < fused_min_n64 && tile_on<double>(H, l)) {
      // a small level: each V(2,2) leg in one region-tile launch -- down (two sweeps,
      // restricted defect, phibar, the coarse level started from it), steps 5-7 on the coarse
      // level, up (the prolonged correction psi - phibar, two sweeps, the norm when asked)
      if (timed) kernel_begin(true);
      tile_down_fas<double>(H.u[l], H.u2[l], H.f[l], H.f[l - 1], pbar[l - 1], H.u[l - 1], n, H.h[l], H.omega, bc, s);
      if (timed) kernel_end("k_tile_leg<double, false, false, false, true>", 3 * cellsT + 3 * cellsT / 8);
      launch_fas_source(pbar[l - 1], H.f[l - 1], n / 2, H.h[l - 1], H.phys[l - 1], s);       // 5
      fas_cycle(H, pbar, l - 1);                                                             // 6
      launch_fas_correction(H.u[l - 1], pbar[l - 1], cells(l - 1), s);                       // 7
      double* npart = want_norm ? part : nullptr;
      if (timed) kernel_begin(true);
      const int np = tile_up<double>(H.u2[l], H.u[l], H.f[l], H.u[l - 1], H.hom, npart, n, 0, 0, H.h[l], H.omega, bc, s);
      if (timed) kernel_end(tile_name<double>(true, npart != nullptr), 3 * cellsT + cellsT / 8);
      if (npart) launch_sum_partials(part, np, scal + 2, s);
      return npart != nullptr;
    }
    const bool streamed = use_fused && H.u2[l] && n >= fused_min_n64;
    // 1: the pre-sweeps; on streamed levels the last one carries steps 2-4 (fused below)
    const int pre = H.npre - done;
    const bool fuse = streamed && pre >= 1;
    double* cur = fas_sweeps(H, l, done > 0 ? H.u2[l] : H.u[l], fuse ? pre - 1 : pre, bc);
    // 2-4 and the coarse start of 6: restricted defect, phibar, u_{l-1} = phibar; algorithmic
    // bytes: u and f read, three coarse arrays written (+ u written with the sweep)
    if (timed) kernel_begin();
    if (fuse) {
      double* oth = cur == H.u[l] ? H.u2[l] : H.u[l];
      fused_sweep_fas_restrict(cur, oth, H.f[l], H.f[l - 1], pbar[l - 1], H.u[l - 1], n, H.h[l], H.omega, bc, s);
      cur = oth;
    } else if (streamed) {
      fused_fas_restrict(cur, H.f[l], H.f[l - 1], pbar[l - 1], H.u[l - 1], n, H.h[l], bc, s);
    } else {
      launch_fas_restrict(cur, H.f[l], H.f[l - 1], pbar[l - 1], H.u[l - 1], n, H.h[l], bc, s);
    }
    if (timed)
      kernel_end(streamed ? fused_fas_restrict_name(fuse) : "k_fas_restrict",
                 (fuse ? 3 * cellsT : 2 * cellsT) + 3 * cellsT / 8);
    launch_fas_source(pbar[l - 1], H.f[l - 1], n / 2, H.h[l - 1], H.phys[l - 1], s);         // 5
    fas_cycle(H, pbar, l - 1);                                                               // 6
    launch_fas_correction(H.u[l - 1], pbar[l - 1], cells(l - 1), s);                         // 7
    // 8-10: the correction obeys the homogeneous conditions (the physical values cancel in
    // psi - phibar); on streamed levels it enters with the first post-sweep, as in Alg. 1
    int post = H.npost;
    if (streamed && post > 0) {
      double* oth = cur == H.u[l] ? H.u2[l] : H.u[l];
      if (timed) kernel_begin();
      fused_prolong_sweep<double>(cur, oth, H.f[l], H.u[l - 1], H.hom, n, H.h[l], H.omega, bc, s);
      if (timed) kernel_end(fused_pass_name<double>(true, 0), 3 * cellsT + cellsT / 8);
      cur = oth;
      --post;
    } else {
      if (timed) kernel_begin();
      launch_prolong<double>(H.u[l - 1], cur, n / 2, H.hom, 0, s);
      // algorithmic bytes: u read and written, the coarse correction read
      if (timed) kernel_end("k_prolong<double, 0>", 2 * cellsT + cellsT / 8);
    }
    cur = fas_sweeps(H, l, cur, post, bc);                                                   // 10
    if (cur != H.u[l]) (void)hipMemcpyAsync(H.u[l], cur, cells(l) * sizeof(double), hipMemcpyDeviceToDevice, s);
    return false;
  }

  // Alg. 2 with FAS in place of the V-cycle.
  // Returns whether the finest level's cycle left the norm of its result in scal[2].
  bool fas_fmg(Hier<double>& H, double* const* pbar) {
    launch_coarsest<double>(H.u[0], H.f[0], H.h[0], H.phys[0], s);
    bool normed = false;
    for (int l = 1; l <= H.L; ++l) {
      launch_prolong<double>(H.u[l - 1], H.u[l], 1 << (l - 1), H.phys[l - 1], 1, s);
      normed = fas_cycle(H, pbar, l, 0, l == H.L);
    }
    return normed;
  }

  // Alg. 2: FMG over all levels with each level's physical description.  norm_top: the
  // finest level's V-cycle may leave the sum of squared defects of its result in scal[2]
  // (returns whether it did).
  template <typename T>
  bool fmg(Hier<T>& H, bool norm_top = false) {
    tail(H, TAIL_FMG, H.phys[H.T_top]);
    bool normed = false;
    for (int l = H.T_top + 1; l <= H.L; ++l) {
      if (Lb >= 0 && l > Lb) {
        blk_prolong<T>(H.u[l - 1], H.u[l], l - Lb, Lb, H.phys[l - 1], 1, s);
        vcycle_blk(H, l, H.phys[l]);
      } else {
        launch_prolong<T>(H.u[l - 1], H.u[l], 1 << (l - 1), H.phys[l - 1], 1, s);
        normed = vcycle(H, l, H.phys[l], false, norm_top && l == H.L);
      }
    }
    return normed;
  }

  // ---- MeshBlock layout (Sec. 3.2): levels above Lb are block levels, Lb and below the root
  // grid and its dense hierarchy.
  int Lb = -1;
  bool timed_top = false;   // kernel timing of the finest block level (V-cycles after FMG)

  template <typename T>
  BlkTune blk_tune(int Lm) const {
    const int key = (sizeof(T) == 8 ? 0 : 1000) + 100 * Lm + Lb;
    auto it = c->blk_tune.find(key);
    if (it != c->blk_tune.end() && blk_tune_valid(it->second, Lm, Lb, sizeof(T), c->lds_per_block)) return it->second;
    return blk_default_tune(Lm, Lb, sizeof(T));
  }

  // npre (or npost) sweeps of block level l, ping-ponging between H.u[l] and H.u2[l], fused
  // S at a time as the schedule says; returns the array holding the result.
  template <typename T>
  T* blk_sweeps(Hier<T>& H, int l, T* cur, int count, const LevelBC& bc) {
    const int Lm = l - Lb;
    const BlkTune t = blk_tune<T>(Lm);
    T* oth = cur == H.u[l] ? H.u2[l] : H.u[l];
    int left = count;
    const bool timed = timed_top && l == H.L && ktiming;
    while (left > 0) {
      BlkTune ti = t;
      ti.S = (t.S == 2 && left >= 2) ? 2 : 1;
      if (!blk_tune_valid(ti, Lm, Lb, sizeof(T), c->lds_per_block)) ti = blk_default_tune(Lm, Lb, sizeof(T));
      if (timed) kernel_begin();
      blk_sweep<T>(cur, oth, H.f[l], Lm, Lb, ti, H.h[l], H.omega, bc, s);
      if (timed)
        kernel_end(std::string("k_blk_sweep<") + (sizeof(T) == 8 ? "double" : "float") + ", " + std::to_string(Lm) +
                       ", " + std::to_string(ti.S) + ">",
                   3.0 * (double)cells(l) * sizeof(T));
      std::swap(cur, oth);
      left -= ti.S;
    }
    return cur;
  }

  // Alg. 1 on block level l: every block at once, one launch per operator; the level below
  // block level Lm = 1 is the root grid (gathered by the restriction, scattered by the
  // prolongation), solved by the dense recursion.
  template <typename T>
  bool blk_zmarch_on(int l) const {
    const int v = c->blk_zmarch[sizeof(T) == 8 ? 0 : 1];
    return (v < 0 ? true : v == 1) && (1 << l) >= (sizeof(T) == 8 ? fused_min_n64 : fused_min_n32);
  }

  // Returns true when want_norm and the sum of squared defects of the result is in scal[2].
  template <typename T>
  bool vcycle_blk(Hier<T>& H, int l, const LevelBC& bc, bool want_norm = false) {
    if (l <= Lb) {
      vcycle(H, l, bc, false, false);
      return false;
    }
    const int Lm = l - Lb;
    const int nl = 1 << l;
    const int vz = c->blk_zmarch[sizeof(T) == 8 ? 0 : 1];
    const bool big = vz != 0 && nl >= march_min<T>() && march_blk_on<T>(H, l, bc);
    if ((big || tile_on<T>(H, l)) && H.npre == 2 && H.npost == 2) {
      // each leg of the block level in one launch over all blocks: the two-sweep streaming
      // passes on the large levels, region tiles below
      const bool timed = timed_top && l == H.L && ktiming;
      const double cellsT = (double)cells(l) * sizeof(T);
      if (l == H.L && down_done) down_done = false;   // queued ahead of the stopping test
      else blk_down_leg<T>(H, l, bc, big, timed);
      vcycle_blk(H, l - 1, H.hom);
      double* npart = want_norm && sizeof(T) == 8 ? part : nullptr;
      if (timed) kernel_begin(true);
      const int np = big ? march_up<T>(H.u2[l], H.u[l], H.f[l], H.u[l - 1], H.hom, npart, nl, H.h[l], H.omega, bc, s, Lm,
                                       aux_of())
                         : tile_up<T>(H.u2[l], H.u[l], H.f[l], H.u[l - 1], H.hom, npart, nl, Lm, Lb, H.h[l], H.omega, bc, s);
      if (timed)
        kernel_end(big ? march_name<T>(true, npart != nullptr, bc, true) : tile_name<T>(true, npart != nullptr, true),
                   3 * cellsT + cellsT / 8);
      if (npart) launch_sum_partials(part, np, scal + 2, s);
      return npart != nullptr;
    }
    if (blk_zmarch_on<T>(l) && H.npre > 0 && H.npost > 0) {
      // streaming passes across block boundaries: one sweep per pass, the restricted defect
      // as its own pass, the prolonged correction entering with the first post-sweep
      const bool timed = timed_top && l == H.L && ktiming;
      const double cellsT = (double)cells(l) * sizeof(T);
      T* cur = H.u[l];
      T* oth = H.u2[l];
      auto pass = [&](const T* ec) {
        if (timed) kernel_begin();
        fused_blk_sweep<T>(cur, oth, H.f[l], ec, H.hom, Lm, Lb, H.h[l], H.omega, bc, s);
        if (timed) kernel_end(fused_blk_pass_name<T>(ec != nullptr, 0), 3 * cellsT + (ec ? cellsT / 8 : 0.0));
        std::swap(cur, oth);
      };
      for (int it = 0; it < H.npre; ++it) pass(nullptr);
      if (timed) kernel_begin();
      fused_blk_defect_restrict<T>(cur, H.f[l], H.f[l - 1], H.u[l - 1], Lm, Lb, H.h[l], bc, s);
      if (timed) kernel_end(fused_blk_pass_name<T>(false, 1), 2 * cellsT + cellsT / 4);
      vcycle_blk(H, l - 1, H.hom);
      pass(H.u[l - 1]);
      for (int it = 1; it < H.npost; ++it) pass(nullptr);
      if (cur != H.u[l]) (void)hipMemcpyAsync(H.u[l], cur, cells(l) * sizeof(T), hipMemcpyDeviceToDevice, s);
      return false;
    }
    T* cur = blk_sweeps(H, l, H.u[l], H.npre, bc);
    blk_defect_restrict<T>(cur, H.f[l], H.f[l - 1], H.u[l - 1], Lm, Lb, H.h[l], bc, s);
    vcycle_blk(H, l - 1, H.hom);
    blk_prolong<T>(H.u[l - 1], cur, Lm, Lb, H.hom, 0, s);
    cur = blk_sweeps(H, l, cur, H.npost, bc);
    if (cur != H.u[l]) (void)hipMemcpyAsync(H.u[l], cur, cells(l) * sizeof(T), hipMemcpyDeviceToDevice, s);
    return false;
  }

  // Source hierarchy f_{l-1} = restriction of f_l (Alg. 2 step 1) in either layout.
  template <typename T>
  void restrict_sources(Hier<T>& H) {
    for (int l = H.L; l >= 1; --l) {
      if (Lb >= 0 && l > Lb) blk_restrict<T, T>(H.f[l], H.f[l - 1], l - Lb, Lb, s);
      else launch_restrict<T, T>(H.f[l], H.f[l - 1], 1 << (l - 1), s);
    }
  }

  // Sum of squared finest-level defects into out (device); optionally the FP32 defect.
  void defect_norm(const double* u, const double* f, float* r32, int n, double h, const LevelBC& bc, double* out) {
    if (Lb >= 0 && n >= kFusedMinN) {
      const int np = fused_blk_defect_norm<double>(u, f, part, ilog2(n) - Lb, Lb, h, bc, s, r32);
      launch_sum_partials(part, np, out, s);
    } else if (Lb >= 0) {
      const int np = blk_defect_norm(u, f, r32, ilog2(n) - Lb, Lb, h, bc, part, s);
      launch_sum_partials(part, np, out, s);
    } else if (n >= kFusedMinN) {
      const int np = fused_defect_norm<double>(u, f, part, n, h, bc, s, r32);
      launch_sum_partials(part, np, out, s);
    } else {
      launch_defect_norm(u, f, r32, n, h, bc, part, out, s);
    }
  }
};

double elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return ms;
}

}  // namespace

// ===================================================================================== ABI

extern "C" {

void mg_default_params(mg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n = 0;
  p->dx = 0;
  p->four_pi_g = 4.0 * M_PI;
  p->mode = MG_MODE_FMG;
  p->npre = 2;
  p->npost = 2;
  p->omega = 1.15;
  p->tol = 1e-10;
  p->max_cycles = 50;
  p->fixed_cycles = 0;
  p->precision = MG_PREC_FP64;
  p->layout = MG_LAYOUT_DENSE;
  p->block_n = 16;
  p->scheme = MG_SCHEME_CS;
}

int mg_ctx_create(mg_ctx** out, int device, size_t hbm_budget) {
  if (!out) return MG_ERR_INVALID_ARG;
  *out = nullptr;
  if (hbm_budget != 0 && hbm_budget < kFixedBytes) return MG_ERR_OOM;
  mg_ctx* c = new mg_ctx();
  c->device = device;
  c->hbm_budget = hbm_budget;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) {
    delete c;
    return MG_ERR_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->lds_per_block = prop.sharedMemPerBlock;
  if (hipMalloc((void**)&c->part, sizeof(double) * kMaxPartials * 32) != hipSuccess ||
      hipMalloc((void**)&c->scal, sizeof(double) * kScal) != hipSuccess ||
      hipHostMalloc((void**)&c->hscal, sizeof(double) * kScal, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->hpub, 2 * sizeof(unsigned long long), hipHostMallocCoherent) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev_setup) != hipSuccess ||
      hipEventCreate(&c->ev_fmg) != hipSuccess) {
    mg_ctx_destroy(c);
    return MG_ERR_DEVICE;
  }
  // the FP64 coarse tail keeps levels <= 16^3 in LDS when the device allows it per block
  c->tail64_top = tail_prepare(c->lds_per_block);
  c->tail_fas = c->tail64_top == 4 && tail_fas_prepare(c->lds_per_block);
  blk_prepare<double>(c->lds_per_block);
  blk_prepare<float>(c->lds_per_block);
  // the static scratch's device address, once per device with the device current (a failure
  // is reported by mg_solve_noalloc, the only user)
  c->static_scratch = static_scratch(device, &c->static_scratch_err);
  // the second stream (default priority) and the fork / join events of the split passes of
  // levels with x or y walls; without them those passes run as one launch
  if (hipStreamCreateWithFlags(&c->aux.s2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->aux.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->aux.join, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    if (c->aux.s2) (void)hipStreamDestroy(c->aux.s2);
    if (c->aux.fork) (void)hipEventDestroy(c->aux.fork);
    c->aux = MarchAux{};
  }
  *out = c;
  return MG_OK;
}

void mg_ctx_destroy(mg_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->ws) (void)hipFree(c->ws);
  if (c->op_scratch) (void)hipFree(c->op_scratch);
  if (c->amr_ws) (void)hipFree(c->amr_ws);
  if (c->part) (void)hipFree(c->part);
  if (c->scal) (void)hipFree(c->scal);
  if (c->hscal) (void)hipHostFree(c->hscal);
  if (c->hpub) (void)hipHostFree(c->hpub);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->aux.s2) (void)hipStreamDestroy(c->aux.s2);
  if (c->aux.fork) (void)hipEventDestroy(c->aux.fork);
  if (c->aux.join) (void)hipEventDestroy(c->aux.join);
  if (c->ev_setup) (void)hipEventDestroy(c->ev_setup);
  if (c->ev_fmg) (void)hipEventDestroy(c->ev_fmg);
  for (auto e : c->ev_cycle) (void)hipEventDestroy(e);
  for (auto e : c->kev) (void)hipEventDestroy(e);
  delete c;
}

const char* mg_last_error(const mg_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t mg_footprint_bytes(const mg_params* p) {
  if (!p || !is_pow2(p->n) || p->n < 2 || p->n > 2048) return 0;
  return make_layout(p->n, p->precision, layout_lb(p), p->scheme == MG_SCHEME_FAS).total + kFixedBytes;
}

int mg_ctx_reserve(mg_ctx* c, const mg_params* p) {
  if (!c || !p) return MG_ERR_INVALID_ARG;
  if (!is_pow2(p->n) || p->n < 2 || p->n > 2048) return fail(c, MG_ERR_INVALID_ARG, "n must be a power of two in [2, 2048]");
  if (p->precision != MG_PREC_FP64 && p->precision != MG_PREC_MIXED) return fail(c, MG_ERR_INVALID_ARG, "bad precision");
  HIP_CHECK(c, hipSetDevice(c->device));
  return ensure_ws(c, make_layout(p->n, p->precision, layout_lb(p), p->scheme == MG_SCHEME_FAS).total);
}

int mg_set_kernel_timing(mg_ctx* c, int on) {
  if (!c) return MG_ERR_INVALID_ARG;
  c->ktiming = on ? 1 : 0;
  return MG_OK;
}

int mg_kernel_timing(const mg_ctx* c, int index, int* launches, double* total_ms, double* bytes_per_launch,
                     char* name, int name_cap) {
  if (!c) return MG_ERR_INVALID_ARG;
  if (index < 0 || index >= (int)c->kstats.size()) return MG_ERR_INVALID_ARG;
  const auto& k = c->kstats[index];
  if (launches) *launches = k.launches;
  if (total_ms) *total_ms = k.ms;
  if (bytes_per_launch) *bytes_per_launch = k.bytes;
  if (name && name_cap > 0) {
    std::strncpy(name, k.name.c_str(), name_cap - 1);
    name[name_cap - 1] = 0;
  }
  return MG_OK;
}

int mg_last_inner(const mg_ctx* c, int* inner_cycles) {
  if (!c || !inner_cycles) return MG_ERR_INVALID_ARG;
  *inner_cycles = c->last_inner;
  return MG_OK;
}

int mg_last_timing(const mg_ctx* c, double* setup_ms, double* fmg_ms, double* cycle_ms, int cap, int* n) {
  if (!c) return MG_ERR_INVALID_ARG;
  if (setup_ms) *setup_ms = c->setup_ms;
  if (fmg_ms) *fmg_ms = c->fmg_ms;
  int m = (int)c->cycle_ms.size();
  if (cycle_ms)
    for (int i = 0; i < std::min(m, cap); ++i) cycle_ms[i] = c->cycle_ms[i];
  if (n) *n = m;
  return MG_OK;
}

}  // extern "C"

namespace {

// Build the per-level physical boundary descriptions in the workspace (Sec. 2.3.6, App. A).
int setup_faces(char* ws, double* part, double* scal, const Layout& y, const mg_params* p, const mg_bc* bc,
                const double* rho, hipStream_t s, LevelBC* phys, LevelBC* hom) {
  const int L = y.L;
  bool any_mp = false;
  for (int f = 0; f < 6; ++f) any_mp |= bc->kind[f] == MG_BC_MULTIPOLE;
  double* mps = scal + kMpoleOff;
  const int Lb = layout_lb(p);
  if (any_mp)
    launch_multipole_moments(rho, p->n, Lb >= 0 ? L - Lb : 0, p->dx, bc->lmax, bc->use_origin, bc->origin, part,
                             mps, s);
  const double G = p->four_pi_g / (4.0 * M_PI);
  for (int l = L; l >= 0; --l) {
    double* fb = reinterpret_cast<double*>(ws + y.faces[l]);
    double* mp_out[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int f = 0; f < 6; ++f) {
      const int k = bc->kind[f];
      double* e = fb + (size_t)f * face_sz(l);
      phys[l].kind[f] = k == MG_BC_MULTIPOLE ? MG_BC_FIXED : k;
      phys[l].b[f] = nullptr;
      if (k == MG_BC_FIXED && bc->fixed_b[f]) {
        if (l == L) launch_face_extend(bc->fixed_b[f], e, 1 << l, s);
        else launch_face_restrict(reinterpret_cast<double*>(ws + y.faces[l + 1]) + (size_t)f * face_sz(l + 1), e,
                                  1 << l, s);
        phys[l].b[f] = e;
      } else if (k == MG_BC_FIXED) {
        // no values: a zero-fixed face, described without an array (ghost = -u, as in the
        // homogeneous descriptions), so the kernels' forms without face values apply
      } else if (k == MG_BC_MULTIPOLE) {
        mp_out[f] = e;
        phys[l].b[f] = e;
      }
    }
    if (any_mp) launch_multipole_faces(mps, bc->lmax, G, 1 << l, p->dx * (double)(1 << (L - l)), p->n * p->dx, mp_out, s);
  }
  for (int f = 0; f < 6; ++f) {
    const int k = bc->kind[f];
    hom->kind[f] = (k == MG_BC_PERIODIC || k == MG_BC_ZERO_GRADIENT) ? k : MG_BC_FIXED;
    hom->b[f] = nullptr;
  }
  // non-finite fixed values are reported with the rho check
  for (int f = 0; f < 6; ++f) {
    if (bc->kind[f] == MG_BC_FIXED && bc->fixed_b[f])
      launch_sum(bc->fixed_b[f], (size_t)p->n * p->n, 2, part, scal + 8 + f, s);
  }
  return MG_OK;
}

}  // namespace

namespace {

// Device memory of one solve: the hierarchy workspace (laid out by make_layout), the
// reduction partials and the device scalars.  `noalloc`: the memory is the library's static
// scratch and the solve allocates nothing (no cycle or kernel timing events either).
struct SolveMem {
  char* ws = nullptr;
  double* part = nullptr;
  double* scal = nullptr;
  bool noalloc = false;
};

// The squared defect norm *dnorm (device) of the cycle just queued on s, for the host's
// stopping test (Sec. 2.3.7), in two steps so that more work can be queued between them.
// post_norm: a one-lane kernel publishes the value with a sequence number (returned) into
// coherent pinned memory; done != nullptr: that event, which ends the cycle's timing, is taken
// from the publishing kernel's own dispatch (an event recorded between kernels would idle the
// device for microseconds; at the publication it costs nothing the host's reply does not
// already).  await_norm: the host spins on the number (waking from a stream synchronisation
// costs tens of microseconds per cycle), polling the stream after 20 ms and every 20 ms from
// then on, so that a failed launch ends the wait with an error; if the stream has finished and the number has not
// arrived, the value is read by a blocking copy and publishing is given up for good (then
// post_norm queues a copy and returns 0).
unsigned long long post_norm(mg_ctx* c, const double* dnorm, hipStream_t s, hipEvent_t done) {
  if (c->pub_ok) {
    const unsigned long long want = ++c->pub_seq;
    launch_publish(dnorm, c->hpub, want, s, done);
    return want;
  }
  if (done) (void)hipEventRecord(done, s);
  (void)hipMemcpyAsync(c->hscal + 2, dnorm, sizeof(double), hipMemcpyDeviceToHost, s);
  return 0;
}

int await_norm(mg_ctx* c, const double* dnorm, hipStream_t s, unsigned long long want, double* out) {
  HIP_CHECK(c, hipGetLastError());
  if (want != 0) {
    // the stream is polled only once the wait has lasted kPollMs, then every kPollMs: a query
    // queues a marker behind the last command, which idles the device for microseconds
    constexpr double kPollMs = 20.0;
    auto t_next = std::chrono::steady_clock::now() + std::chrono::duration<double, std::milli>(kPollMs);
    for (unsigned spin = 1;; ++spin) {
      if (__atomic_load_n(c->hpub + 1, __ATOMIC_ACQUIRE) == want) {
        *out = __builtin_bit_cast(double, __atomic_load_n(c->hpub, __ATOMIC_RELAXED));
        return MG_OK;
      }
      if ((spin & 1023u) == 0 && std::chrono::steady_clock::now() >= t_next) {
        t_next = std::chrono::steady_clock::now() + std::chrono::duration<double, std::milli>(kPollMs);
        const hipError_t q = hipStreamQuery(s);
        if (q == hipErrorNotReady) continue;
        HIP_CHECK(c, q);
        if (__atomic_load_n(c->hpub + 1, __ATOMIC_ACQUIRE) == want) {
          *out = __builtin_bit_cast(double, __atomic_load_n(c->hpub, __ATOMIC_RELAXED));
          return MG_OK;
        }
        c->pub_ok = false;
        HIP_CHECK(c, hipMemcpyAsync(c->hscal + 2, dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
        break;
      }
      __builtin_ia32_pause();
    }
  }
  HIP_CHECK(c, hipStreamSynchronize(s));
  *out = c->hscal[2];
  return MG_OK;
}

int solve_impl(mg_ctx* c, const mg_params* p, const mg_bc* bc, const double* rho, double* phi, double* hist,
               int* n_hist, hipStream_t s, const Layout& y, const SolveMem& mem) {
  const int Lb = layout_lb(p);
  const bool fas = p->scheme == MG_SCHEME_FAS;
  char* const ws = mem.ws;
  double* const part = mem.part;
  double* const scal = mem.scal;
  const int ktiming = mem.noalloc ? 0 : c->ktiming;
  if (!mem.noalloc) {
    for (auto e : c->kev) (void)hipEventDestroy(e);
    c->kev.clear();
    c->kev_id.clear();
    c->kstats.clear();
  }

  const int L = y.L;
  const size_t n3 = cells(L);
  bool gauge_free = true;
  for (int f = 0; f < 6; ++f)
    if (bc->kind[f] == MG_BC_FIXED || bc->kind[f] == MG_BC_MULTIPOLE) gauge_free = false;
  const bool mixed = y.mixed;
  int tail_max = mixed ? 4 : c->tail64_top;
  if (c->tail_top[mixed ? 1 : 0] > 0) tail_max = std::min(tail_max, c->tail_top[mixed ? 1 : 0]);
  tail_max = std::min(tail_max, Lb >= 0 ? Lb : 99);

  HIP_CHECK(c, hipEventRecord(c->ev0, s));
  launch_zero(scal, sizeof(double) * kScal, s);

  // ---- source (eq. poisson, f = 4 pi G rho; mean removed when gauge-free, Sec. 2.3.6)
  double* f64L = reinterpret_cast<double*>(ws + y.f64L);
  float* f32L = mixed ? reinterpret_cast<float*>(ws + y.f32[L]) : nullptr;
  // (gauge-free: the source kernel reads the sum of rho from scal[0] and shifts by the mean)
  launch_sum(rho, n3, 0, part, scal + 0, s);
  launch_source(rho, f64L, f32L, n3, p->four_pi_g, gauge_free ? scal + 0 : nullptr, part, scal + 1, s);

  LevelBC phys[16], hom;
  setup_faces(ws, part, scal, y, p, bc, rho, s, phys, &hom);

  Solver S{c, s, true};
  S.part = part;
  S.scal = scal;
  S.ktiming = ktiming;
  S.Lb = Lb;
  if (c->fused_min_n[0] > 0) S.fused_min_n64 = c->fused_min_n[0];
  if (c->fused_min_n[1] > 0) S.fused_min_n32 = c->fused_min_n[1];
  Hier<double> H64;
  Hier<float> H32;
  auto fill_common = [&](auto& H, int tail_top) {
    H.L = L;
    H.T_top = std::min(L, tail_top);
    H.npre = p->npre;
    H.npost = p->npost;
    H.omega = p->omega;
    H.hom = hom;
    for (int l = 0; l <= L; ++l) {
      H.h[l] = p->dx * (double)(1LL << (L - l));
      H.phys[l] = phys[l];
    }
  };
  if (!mixed) {
    fill_common(H64, tail_max);
    for (int l = 0; l < L; ++l) {
      H64.u[l] = reinterpret_cast<double*>(ws + y.u64[l]);
      H64.f[l] = reinterpret_cast<double*>(ws + y.f64[l]);
    }
    H64.u[L] = phi;
    H64.f[L] = f64L;
    for (int l = 0; l <= L; ++l)
      H64.u2[l] = y.u2[l] == (size_t)-1 ? nullptr : reinterpret_cast<double*>(ws + y.u2[l]);
    S.restrict_sources(H64);
  } else {
    fill_common(H32, tail_max);
    for (int l = 0; l <= L; ++l) {
      H32.u[l] = reinterpret_cast<float*>(ws + y.u32[l]);
      H32.f[l] = reinterpret_cast<float*>(ws + y.f32[l]);
      H32.u2[l] = y.u2[l] == (size_t)-1 ? nullptr : reinterpret_cast<float*>(ws + y.u2[l]);
    }
    S.restrict_sources(H32);
  }
  HIP_CHECK(c, hipEventRecord(c->ev_setup, s));

  // ---- FMG sweep (Alg. 2) or the caller's initial guess
  double* pbar[16] = {nullptr};
  if (fas)
    for (int l = 0; l < L; ++l) pbar[l] = reinterpret_cast<double*>(ws + y.pbar[l]);
  bool fmg_normed = false;
  if (p->mode == MG_MODE_FMG) {
    if (fas) {
      fmg_normed = S.fas_fmg(H64, pbar);
    } else if (!mixed) {
      // the finest level's FMG V-cycle takes the norm of its result when its up pass can
      fmg_normed = S.fmg(H64, S.march_on<double>(H64, L, phys[L]) ||
                                  (p->n < S.fused_min_n64 && S.tile_on<double>(H64, L)));
    } else {
      S.fmg(H32);
      launch_f32_to_f64(H32.u[L], phi, n3, s);
    }
  }
  // ---- residual of the start (Sec. 2.3.7); mixed: also its FP32 copy as the inner RHS.  FP64
  // on the fused path: taken by the head pass, which is also the first sweep of V-cycle 1
  // (of the FAS cycle 1 with the Full Approximation Scheme)
  const bool head_mode = !mixed && Lb < 0 && S.head_possible(H64);
  if (head_mode) S.head(H64, phys[L]);
  else if (!fmg_normed) S.defect_norm(phi, f64L, mixed ? H32.f[L] : nullptr, p->n, p->dx, phys[L], scal + 2);
  HIP_CHECK(c, hipEventRecord(c->ev_fmg, s));
  HIP_CHECK(c, hipMemcpyAsync(c->hscal, scal, sizeof(double) * 16, hipMemcpyDeviceToHost, s));
  HIP_CHECK(c, hipStreamSynchronize(s));
  bool finite = std::isfinite(c->hscal[0]) && std::isfinite(c->hscal[1]);
  for (int f = 0; f < 6; ++f) finite = finite && c->hscal[8 + f] == 0.0;
  if (!finite) return fail(c, MG_ERR_NONFINITE, "non-finite values in rho or fixed boundary values");
  const double rms_f = std::sqrt(c->hscal[1] / (double)n3);
  auto rel = [&](double sumsq) {
    const double rd = std::sqrt(sumsq / (double)n3);
    return rms_f > 0 ? rd / rms_f : rd;
  };
  double r = rel(c->hscal[2]);
  int nh = 0;
  hist[nh++] = r;

  // ---- V-cycles until the stopping test (Sec. 2.3.7)
  const int ncyc = p->fixed_cycles > 0 ? p->fixed_cycles : p->max_cycles;
  // per-cycle timing events (created once, reused; none in the allocation-free form)
  while (!mem.noalloc && (int)c->ev_cycle.size() < ncyc) {
    hipEvent_t e;
    HIP_CHECK(c, hipEventCreate(&e));
    c->ev_cycle.push_back(e);
  }
  const bool cyc_timed = !mem.noalloc;
  int status = p->fixed_cycles > 0 ? MG_OK : MG_NOT_CONVERGED;
  int slow = 0, done_cycles = 0;
  double* phi_cur = phi;     // mixed mode alternates phi with its ping-pong partner
  double* phi_oth = y.phi2 == (size_t)-1 ? nullptr : reinterpret_cast<double*>(ws + y.phi2);
  // mixed: FP32 V-cycles per outer step -- the "inner" setting, else (to a tolerance) as many
  // as the residual contraction per V-cycle seen so far says are still needed, at most 3 (one
  // in fixed-cycle runs).  The contraction is taken 1.5 times as slow as seen (it slows as the
  // iterate converges): one V-cycle too many costs less than another outer step with its FP64
  // update pass.  The count of the whole solve is kept for mg_last_inner
  c->last_inner = 0;
  double rho_est = 0.1;
  // first legs queued ahead of the stopping test: FP64 correction-scheme cycles (not in head
  // mode, whose head pass already overlaps the test); rho_seen = the last cycle's contraction
  const bool ahead_ok = !mixed && !fas && !head_mode;
  double rho_seen = 0.1;
  if (p->fixed_cycles > 0 || r > p->tol) {
    for (int cyc = 0; cyc < ncyc; ++cyc) {
      S.timed_top = true;
      int inner = 1;
      if (mixed && !(Lb < 0 && L == H32.T_top)) {
        if (c->inner > 0) {
          inner = c->inner;
        } else if (p->fixed_cycles <= 0 && r > p->tol) {
          const double m = std::ceil(std::log(p->tol / r) / std::log(std::min(0.5, 1.5 * rho_est)));
          inner = (int)std::min(3.0, std::max(1.0, m));
        }
      }
      if (fas) {
        // as below: the head pass of the next cycle measures this cycle's result (or the
        // two-sweep up pass does)
        const bool normed = S.fas_cycle(H64, pbar, L, head_mode ? 1 : 0, !head_mode);
        S.head_done = false;
        if (head_mode && cyc + 1 < ncyc) S.head(H64, phys[L]);
        else if (!normed) S.defect_norm(phi, f64L, nullptr, p->n, p->dx, phys[L], scal + 2);
      } else if (head_mode) {
        // the rest of this V-cycle (its first sweep ran in the head pass), then the head of the
        // next one, which measures this cycle's result; after the last allowed cycle the
        // residual alone (a head's sweep would be discarded)
        S.head_done = true;
        S.vcycle(H64, L, phys[L], true, false);
        if (cyc + 1 < ncyc) S.head(H64, phys[L]);
        else S.defect_norm(phi, f64L, nullptr, p->n, p->dx, phys[L], scal + 2);
      } else if (!mixed && Lb >= 0) {
        if (!S.vcycle_blk(H64, L, phys[L], true)) S.defect_norm(phi, f64L, nullptr, p->n, p->dx, phys[L], scal + 2);
      } else if (mixed && Lb >= 0) {
        launch_zero(H32.u[L], n3 * sizeof(float), s);
        for (int k = 0; k < inner; ++k) S.vcycle_blk(H32, L, hom);
        launch_add_f32(phi, H32.u[L], n3, s);
        S.defect_norm(phi, f64L, H32.f[L], p->n, p->dx, phys[L], scal + 2);
      } else if (!mixed) {
        const bool normed = S.vcycle(H64, L, phys[L], true, true);
        if (!normed) S.defect_norm(phi, f64L, nullptr, p->n, p->dx, phys[L], scal + 2);
      } else {
        // defect correction: e32 solves L e = r32 from zero with homogeneous conditions
        if (L == H32.T_top) {
          S.tail(H32, 0, hom);
        } else {
          // the correction starts from zero: the first sweep does not read it (or the
          // V-cycle clears it when its first pass cannot skip the read)
          S.zero_start = true;
          for (int k = 0; k < inner; ++k) {
            S.vcycle(H32, L, hom, true, false);
            S.zero_start = false;
          }
        }
        if (phi_oth) {
          // phi += e and the FP64 defect (with its FP32 copy and norm) in one streaming pass
          const int np = fused_mixed_update_defect(phi_cur, phi_oth, H32.u[L], f64L, H32.f[L], part, p->n, p->dx,
                                                   phys[L], s);
          launch_sum_partials(part, np, scal + 2, s);
          std::swap(phi_cur, phi_oth);
        } else {
          launch_add_f32(phi, H32.u[L], n3, s);
          S.defect_norm(phi, f64L, H32.f[L], p->n, p->dx, phys[L], scal + 2);
        }
      }
      const unsigned long long want = post_norm(c, scal + 2, s, cyc_timed ? c->ev_cycle[cyc] : nullptr);
      // the next cycle's first leg is queued before this cycle's norm is read when that leg
      // reads u only and another cycle will run: always with a fixed cycle count, and when the
      // tolerance is still at least 4x past what this cycle reaches at the contraction seen so
      // far (had the solve stopped after all, that leg's results go unused)
      if (ahead_ok && cyc + 1 < ncyc && (p->fixed_cycles > 0 || 0.25 * rho_seen * r > p->tol))
        (void)S.down_ahead(H64, phys[L]);
      double d2 = 0.0;
      if (const int st = await_norm(c, scal + 2, s, want, &d2); st != MG_OK) return st;
      const double rn = rel(d2);
      if (r > 0 && rn > 0) rho_seen = std::min(1.0, rn / r);
      hist[nh++] = rn;
      ++done_cycles;
      if (mixed) {
        c->last_inner += inner;
        if (r > 0 && rn > 0 && rn < r) rho_est = std::min(0.5, std::max(0.01, std::pow(rn / r, 1.0 / inner)));
      }
      if (p->fixed_cycles > 0) { r = rn; continue; }
      slow = rn > 0.9 * r ? slow + 1 : 0;
      r = rn;
      if (r <= p->tol) { status = MG_OK; break; }
      if (slow >= 2) { status = MG_STALLED; break; }
    }
  } else {
    status = MG_OK;
  }
  if (S.down_done) {   // a leg queued ahead of a test that then stopped the solve: unused
    S.down_done = false;
    S.drop_ahead_timing();
  }
  *n_hist = nh;
  if (phi_cur != phi) HIP_CHECK(c, hipMemcpyAsync(phi, phi_cur, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));

  // ---- gauge (Sec. 2.3.6): zero mean potential when no face fixes the zero point
  if (gauge_free) {
    launch_sum(phi, n3, 0, part, scal + 3, s);
    launch_sub_mean(phi, n3, scal + 3, s);
  }
  HIP_CHECK(c, hipStreamSynchronize(s));
  HIP_CHECK(c, hipGetLastError());

  // ---- timing
  c->setup_ms = elapsed(c->ev0, c->ev_setup);
  c->fmg_ms = elapsed(c->ev_setup, c->ev_fmg);
  c->cycle_ms.clear();
  hipEvent_t prev = c->ev_fmg;
  for (int cyc = 0; cyc < done_cycles && cyc_timed; ++cyc) {
    c->cycle_ms.push_back(elapsed(prev, c->ev_cycle[cyc]));
    prev = c->ev_cycle[cyc];
  }
  if (ktiming) {
    for (size_t q = 0; q + 1 < c->kev.size(); q += 2) {
      auto& k = c->kstats[c->kev_id[q / 2]];
      k.ms += elapsed(c->kev[q], c->kev[q + 1]);
      k.launches += 1;
    }
  }
  return status;
}

}  // namespace

extern "C" int mg_solve(mg_ctx* c, const mg_params* p, const mg_bc* bc, const double* rho, double* phi, double* hist,
                        int* n_hist, void* stream) {
  if (!c) return MG_ERR_INVALID_ARG;
  if (n_hist) *n_hist = 0;
  int st = validate(c, p, bc);
  if (st != MG_OK) return st;
  if (!rho || !phi || !hist || !n_hist) return fail(c, MG_ERR_INVALID_ARG, "null rho/phi/hist/n_hist");
  HIP_CHECK(c, hipSetDevice(c->device));
  const Layout y = make_layout(p->n, p->precision, layout_lb(p), p->scheme == MG_SCHEME_FAS);
  st = ensure_ws(c, y.total);
  if (st != MG_OK) return st;
  SolveMem mem;
  mem.ws = c->ws;
  mem.part = c->part;
  mem.scal = c->scal;
  return solve_impl(c, p, bc, rho, phi, hist, n_hist, reinterpret_cast<hipStream_t>(stream), y, mem);
}

extern "C" int mg_solve_noalloc(mg_ctx* c, const mg_params* p, const mg_bc* bc, const double* rho, double* phi,
                                double* hist, int* n_hist, void* stream) {
  if (!c) return MG_ERR_INVALID_ARG;
  if (n_hist) *n_hist = 0;
  int st = validate(c, p, bc);
  if (st != MG_OK) return st;
  if (!rho || !phi || !hist || !n_hist) return fail(c, MG_ERR_INVALID_ARG, "null rho/phi/hist/n_hist");
  if (!c->static_scratch)
    return fail(c, MG_ERR_DEVICE, std::string("static scratch address: ") + hipGetErrorString(c->static_scratch_err));
  const Layout y = make_layout(p->n, p->precision, layout_lb(p), p->scheme == MG_SCHEME_FAS);
  // the static scratch holds the device scalars, the reduction partials and the workspace
  const size_t scal_bytes = align_up(sizeof(double) * kScal);
  const size_t part_bytes = align_up(sizeof(double) * kMaxPartials * 32);
  const size_t need = scal_bytes + part_bytes + y.total;
  if (need > kStaticScratchBytes)
    return fail(c, MG_ERR_OOM, "mg_solve_noalloc: this solve needs " + std::to_string(need) +
                                   " bytes of scratch; the static scratch holds " +
                                   std::to_string(kStaticScratchBytes) + " (every precision and layout up to n = 128)");
  HIP_CHECK(c, hipSetDevice(c->device));
  SolveMem mem;
  mem.scal = reinterpret_cast<double*>(c->static_scratch);
  mem.part = reinterpret_cast<double*>(c->static_scratch + scal_bytes);
  mem.ws = c->static_scratch + scal_bytes + part_bytes;
  mem.noalloc = true;
  return solve_impl(c, p, bc, rho, phi, hist, n_hist, reinterpret_cast<hipStream_t>(stream), y, mem);
}

extern "C" int mg_solve_simple(mg_ctx* c, int n, const double* rho, int bc_kind, double dx, double tol, double* phi,
                               double* hist, int* n_hist, void* stream) {
  if (!c) return MG_ERR_INVALID_ARG;
  if (n_hist) *n_hist = 0;
  if (bc_kind < MG_BC_PERIODIC || bc_kind > MG_BC_MULTIPOLE) return fail(c, MG_ERR_INVALID_ARG, "bad face kind");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(c, MG_ERR_INVALID_ARG, "tol must be positive");
  mg_params p;
  mg_default_params(&p);
  p.n = n;
  p.dx = dx;
  p.tol = tol;
  mg_bc bc;
  std::memset(&bc, 0, sizeof(bc));
  for (int f = 0; f < 6; ++f) bc.kind[f] = bc_kind;
  bc.lmax = 4;
  return mg_solve(c, &p, &bc, rho, phi, hist, n_hist, stream);
}

// ============================================================== autotuner

namespace {

template <typename T>
int autotune_blocks(mg_ctx* c, const mg_params* p, int Lb, int reps) {
  const int L = ilog2(p->n);
  const size_t cellsL = cells(L);
  // u (two), f, and the coarse source and correction of the finest block level
  T* buf[4] = {nullptr, nullptr, nullptr, nullptr};
  const size_t sz[4] = {cellsL, cellsL, cellsL, cellsL / 4};
  if (over_budget(c, (3 * cellsL + cellsL / 4) * sizeof(T), 0))
    return fail(c, MG_ERR_OOM, "autotune scratch exceeds the HBM budget");
  for (int q = 0; q < 4; ++q)
    if (hipMalloc((void**)&buf[q], sz[q] * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      for (auto& b : buf)
        if (b) (void)hipFree(b);
      return fail(c, MG_ERR_OOM, "autotune scratch allocation failed");
    }
  hipStream_t s = nullptr;
  HIP_CHECK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  for (int q = 0; q < 4; ++q) HIP_CHECK(c, hipMemsetAsync(buf[q], 0, sz[q] * sizeof(T), s));
  hipEvent_t e0, e1;
  HIP_CHECK(c, hipEventCreate(&e0));
  HIP_CHECK(c, hipEventCreate(&e1));
  LevelBC bc;
  for (int f = 0; f < 6; ++f) { bc.kind[f] = BC_PERIODIC; bc.b[f] = nullptr; }
  for (int l = Lb + 1; l <= L; ++l) {
    const int Lm = l - Lb;
    const double h = p->dx * (double)(1LL << (L - l));
    BlkTune best = blk_default_tune(Lm, Lb, sizeof(T));
    double best_ms = 1e30;
    for (int S = 1; S <= 2; ++S)
      for (int threads : {256, 512, 1024})
        for (int G = 1; G <= 256; G *= 2) {
          const BlkTune t{threads, G, S};
          if (!blk_tune_valid(t, Lm, Lb, sizeof(T), c->lds_per_block)) continue;
          const int tw = (1 << Lm) + 4 * S;
          if (G > 1 && (size_t)G * tw * tw * tw > 40000) continue;   // beyond ~4 workgroups' worth per CU
          blk_sweep<T>(buf[0], buf[1], buf[2], Lm, Lb, t, h, p->omega, bc, s);
          HIP_CHECK(c, hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) blk_sweep<T>(buf[r & 1], buf[(r + 1) & 1], buf[2], Lm, Lb, t, h, p->omega, bc, s);
          HIP_CHECK(c, hipEventRecord(e1, s));
          HIP_CHECK(c, hipEventSynchronize(e1));
          HIP_CHECK(c, hipGetLastError());
          const double ms = elapsed(e0, e1) / (reps * S);   // per sweep
          if (ms < best_ms) { best_ms = ms; best = t; }
        }
    c->blk_tune[(sizeof(T) == 8 ? 0 : 1000) + 100 * Lm + Lb] = best;
    if (l == L && p->npre == 2 && p->npost == 2 && (1 << l) >= march_min_n<T>(c) && blk_march_fits(l)) {
      // V(2,2) on the finest block level: both legs as the two-sweep streaming passes across
      // blocks against the four halo-tile sweeps alone (a lower bound on that schedule)
      T* fc = buf[3];
      T* uc = buf[3] + cellsL / 8;
      LevelBC hom = bc;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) {
        march_down<T>(buf[0], buf[1], buf[2], fc, uc, 1 << l, h, p->omega, bc, s, Lm);
        (void)march_up<T>(buf[1], buf[0], buf[2], uc, hom, nullptr, 1 << l, h, p->omega, bc, s, Lm);
      }
      (void)hipEventRecord(e1, s);
      HIP_CHECK(c, hipEventSynchronize(e1));
      HIP_CHECK(c, hipGetLastError());
      const double t_m = elapsed(e0, e1) / reps;
      c->blk_zmarch[sizeof(T) == 8 ? 0 : 1] = t_m < 4.0 * best_ms ? 1 : 0;
    } else if (l == L && (1 << l) >= kFusedDefaultMinN) {
      // the finest block level: halo-tile sweeps against the streaming passes across blocks
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r)
        fused_blk_sweep<T>(buf[r & 1], buf[(r + 1) & 1], buf[2], nullptr, bc, Lm, Lb, h, p->omega, bc, s);
      (void)hipEventRecord(e1, s);
      HIP_CHECK(c, hipEventSynchronize(e1));
      const double t_z = elapsed(e0, e1) / reps;
      c->blk_zmarch[sizeof(T) == 8 ? 0 : 1] = t_z < best_ms ? 1 : 0;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  for (auto& b : buf) (void)hipFree(b);
  return MG_OK;
}

// Dense layout: for each fused level, time the restricted defect fused into the last
// pre-smoothing pass against a plain sweep followed by the defect-only pass (and, for the FP64
// finest level, the same for the norm), and keep the faster schedule.
template <typename T>
int autotune_dense(mg_ctx* c, const mg_params* p, int reps) {
  const int L = ilog2(p->n);
  const size_t cellsL = cells(L);
  T* buf[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t sz[5] = {cellsL, cellsL, cellsL, cellsL / 8, cellsL / 8};
  if (over_budget(c, (3 * cellsL + cellsL / 4) * sizeof(T), 0))
    return fail(c, MG_ERR_OOM, "autotune scratch exceeds the HBM budget");
  for (int q = 0; q < 5; ++q)
    if (hipMalloc((void**)&buf[q], sz[q] * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      for (auto& b : buf)
        if (b) (void)hipFree(b);
      return fail(c, MG_ERR_OOM, "autotune scratch allocation failed");
    }
  hipStream_t s = nullptr;
  HIP_CHECK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  for (int q = 0; q < 5; ++q) HIP_CHECK(c, hipMemsetAsync(buf[q], 0, sz[q] * sizeof(T), s));
  hipEvent_t e0, e1;
  HIP_CHECK(c, hipEventCreate(&e0));
  HIP_CHECK(c, hipEventCreate(&e1));
  LevelBC bc;
  for (int f = 0; f < 6; ++f) { bc.kind[f] = BC_PERIODIC; bc.b[f] = nullptr; }
  auto time_it = [&](auto&& body) -> double {
    body();
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) body();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    return elapsed(e0, e1) / reps;
  };
  for (int l = ilog2(kFusedMinN); l <= L; ++l) {
    const int n = 1 << l;
    const double h = p->dx * (double)(1LL << (L - l));
    const double t_fused = time_it([&] {
      fused_sweep_defect<T>(buf[0], buf[1], buf[2], buf[3], buf[4], n, h, p->omega, bc, s);
    });
    const double t_split = time_it([&] {
      fused_sweep<T>(buf[0], buf[1], buf[2], n, h, p->omega, bc, s);
      fused_defect_restrict<T>(buf[1], buf[2], buf[3], buf[4], n, h, bc, s);
    });
    int split = t_split < t_fused ? 1 : 0;
    if (sizeof(T) == 8 && l == L) {
      const double t_nf = time_it([&] {
        (void)fused_sweep_norm<T>(buf[0], buf[1], buf[2], c->part, n, h, p->omega, bc, s);
      });
      const double t_ns = time_it([&] {
        fused_sweep<T>(buf[0], buf[1], buf[2], n, h, p->omega, bc, s);
        (void)fused_defect_norm<T>(buf[1], buf[2], c->part, n, h, bc, s);
      });
      if (t_ns < t_nf) split |= 2;
    }
    if (l == L) {
      // sweep fusion: two one-sweep passes against one temporally blocked two-sweep pass
      const double t_one = time_it([&] {
        fused_sweep<T>(buf[0], buf[1], buf[2], n, h, p->omega, bc, s);
        fused_sweep<T>(buf[1], buf[0], buf[2], n, h, p->omega, bc, s);
      });
      const double t_two = time_it([&] {
        tb_sweeps<T>(buf[0], buf[1], buf[2], nullptr, bc, 2, n, h, p->omega, bc, s);
      });
      c->tblock[sizeof(T) == 8 ? 0 : 1] = t_two < t_one ? 1 : 0;
    }
    HIP_CHECK(c, hipGetLastError());
    c->pass_split[(sizeof(T) == 8 ? 0 : 1000) + l] = split;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  for (auto& b : buf) (void)hipFree(b);
  return MG_OK;
}

}  // namespace

extern "C" {

int mg_autotune(mg_ctx* c, const mg_params* p, int reps) {
  if (!c || !p) return MG_ERR_INVALID_ARG;
  mg_bc bc;
  std::memset(&bc, 0, sizeof(bc));
  int st = validate(c, p, &bc);
  if (st != MG_OK) return st;
  if (reps < 1 || reps > 1000) return fail(c, MG_ERR_INVALID_ARG, "reps in 1..1000");
  HIP_CHECK(c, hipSetDevice(c->device));
  const int Lb = layout_lb(p);
  if (Lb < 0) {
    if (p->n < kFusedMinN) return MG_OK;
    return p->precision == MG_PREC_MIXED ? autotune_dense<float>(c, p, reps) : autotune_dense<double>(c, p, reps);
  }
  st = p->precision == MG_PREC_MIXED ? autotune_blocks<float>(c, p, Lb, reps) : autotune_blocks<double>(c, p, Lb, reps);
  return st;
}

int mg_tuning_get(const mg_ctx* c, char* buf, int cap) {
  if (!c) return MG_ERR_INVALID_ARG;
  std::ostringstream o;
  for (const auto& kv : c->blk_tune) {
    const int key = kv.first;
    o << "blk " << (key >= 1000 ? "fp32" : "fp64") << " " << (key % 1000) / 100 << " " << key % 100 << " "
      << kv.second.threads << " " << kv.second.G << " " << kv.second.S << "\n";
  }
  for (const auto& kv : c->pass_split)
    o << "pass " << (kv.first >= 1000 ? "fp32" : "fp64") << " " << kv.first % 1000 << " " << kv.second << "\n";
  for (int q = 0; q < 2; ++q) {
    if (c->fused_min_n[q] > 0) o << "fusedmin " << (q ? "fp32" : "fp64") << " " << c->fused_min_n[q] << "\n";
    if (c->tail_top[q] > 0) o << "tail " << (q ? "fp32" : "fp64") << " " << c->tail_top[q] << "\n";
    if (c->tblock[q] >= 0) o << "tb " << (q ? "fp32" : "fp64") << " " << c->tblock[q] << "\n";
    if (c->blk_zmarch[q] >= 0) o << "blkz " << (q ? "fp32" : "fp64") << " " << c->blk_zmarch[q] << "\n";
    if (c->march[q] >= 0) o << "march " << (q ? "fp32" : "fp64") << " " << c->march[q] << "\n";
    if (c->tile[q] >= 0) o << "tile " << (q ? "fp32" : "fp64") << " " << c->tile[q] << "\n";
  }
  if (c->split >= 0) o << "split fp64 " << c->split << "\n";
  if (c->inner > 0) o << "inner fp32 " << c->inner << "\n";
  const std::string t = o.str();
  if (buf && cap > 0) {
    std::strncpy(buf, t.c_str(), (size_t)cap - 1);
    buf[cap - 1] = 0;
  }
  return (int)t.size() + 1;
}

int mg_tuning_set(mg_ctx* c, const char* text) {
  if (!c || !text) return MG_ERR_INVALID_ARG;
  std::istringstream in(text);
  std::string line;
  std::map<int, BlkTune> add;
  std::map<int, int> add_pass;
  std::vector<std::pair<int, int>> add_misc;
  while (std::getline(in, line)) {
    if (line.empty()) continue;
    std::istringstream ls(line);
    std::string tag, prec;
    if (line.rfind("split ", 0) == 0) {
      int v;
      if (!(ls >> tag >> prec >> v) || prec != "fp64" || v < 0 || v > 1)
        return fail(c, MG_ERR_INVALID_ARG, "bad tuning line: " + line);
      add_misc.push_back({12, v});
      continue;
    }
    if (line.rfind("inner ", 0) == 0) {
      int v;
      if (!(ls >> tag >> prec >> v) || prec != "fp32" || v < 1 || v > 4)
        return fail(c, MG_ERR_INVALID_ARG, "bad tuning line: " + line);
      add_misc.push_back({13, v});
      continue;
    }
    if (line.rfind("tb ", 0) == 0 || line.rfind("blkz ", 0) == 0 || line.rfind("march ", 0) == 0 ||
        line.rfind("tile ", 0) == 0) {
      int v;
      const int vmax = line.rfind("march ", 0) == 0 ? 2 : 1;
      if (!(ls >> tag >> prec >> v) || (prec != "fp64" && prec != "fp32") || v < 0 || v > vmax)
        return fail(c, MG_ERR_INVALID_ARG, "bad tuning line: " + line);
      add_misc.push_back({(tag == "tb" ? 4 : tag == "blkz" ? 6 : tag == "march" ? 8 : 10) + (prec == "fp64" ? 0 : 1), v});
      continue;
    }
    if (line.rfind("fusedmin ", 0) == 0 || line.rfind("tail ", 0) == 0) {
      int v;
      if (!(ls >> tag >> prec >> v) || (prec != "fp64" && prec != "fp32"))
        return fail(c, MG_ERR_INVALID_ARG, "bad tuning line: " + line);
      const int q = prec == "fp64" ? 0 : 1;
      if (tag == "fusedmin") {
        if (!is_pow2(v) || v < kFusedMinN || v > 4096) return fail(c, MG_ERR_INVALID_ARG, "fusedmin: power of two >= 64");
        add_misc.push_back({q, v});
      } else {
        if (v < 1 || v > 4) return fail(c, MG_ERR_INVALID_ARG, "tail: level 1..4");
        add_misc.push_back({2 + q, v});
      }
      continue;
    }
    if (line.rfind("pass ", 0) == 0) {
      int l, split;
      if (!(ls >> tag >> prec >> l >> split) || (prec != "fp64" && prec != "fp32") || l < 0 || l > 11 || split < 0 ||
          split > 3)
        return fail(c, MG_ERR_INVALID_ARG, "bad tuning line: " + line);
      add_pass[(prec == "fp64" ? 0 : 1000) + l] = split;
      continue;
    }
    int Lm, Lb, threads, G, S;
    if (!(ls >> tag >> prec >> Lm >> Lb >> threads >> G >> S) || tag != "blk" || (prec != "fp64" && prec != "fp32"))
      return fail(c, MG_ERR_INVALID_ARG, "bad tuning line: " + line);
    const BlkTune t{threads, G, S};
    if (Lb < 0 || Lb > 10 || !blk_tune_valid(t, Lm, Lb, prec == "fp64" ? 8 : 4, c->lds_per_block))
      return fail(c, MG_ERR_INVALID_ARG, "invalid schedule: " + line);
    add[(prec == "fp64" ? 0 : 1000) + 100 * Lm + Lb] = t;
  }
  for (const auto& kv : add) c->blk_tune[kv.first] = kv.second;
  for (const auto& kv : add_pass) c->pass_split[kv.first] = kv.second;
  for (const auto& kv : add_misc) {
    if (kv.first < 2) c->fused_min_n[kv.first] = kv.second;
    else if (kv.first < 4) c->tail_top[kv.first - 2] = kv.second;
    else if (kv.first < 6) c->tblock[kv.first - 4] = kv.second;
    else if (kv.first < 8) c->blk_zmarch[kv.first - 6] = kv.second;
    else if (kv.first < 10) c->march[kv.first - 8] = kv.second;
    else if (kv.first < 12) c->tile[kv.first - 10] = kv.second;
    else if (kv.first == 12) c->split = kv.second;
    else c->inner = kv.second;
  }
  return MG_OK;
}

}  // extern "C"

// ============================================================== operator entry points

namespace {
int op_prologue(mg_ctx* c, int n) {
  if (!c) return MG_ERR_INVALID_ARG;
  if (!is_pow2(n) || n > 2048) return fail(c, MG_ERR_INVALID_ARG, "n must be a power of two <= 2048");
  HIP_CHECK(c, hipSetDevice(c->device));
  return MG_OK;
}
int op_epilogue(mg_ctx* c) {
  HIP_CHECK(c, hipGetLastError());
  return MG_OK;
}
int op_scratch(mg_ctx* c, size_t bytes, double** out) {
  if (bytes > c->op_scratch_cap) {
    if (over_budget(c, bytes, c->op_scratch_cap))
      return fail(c, MG_ERR_OOM, "operator scratch exceeds the context's HBM budget");
    if (c->op_scratch) {
      HIP_CHECK(c, hipDeviceSynchronize());
      HIP_CHECK(c, hipFree(c->op_scratch));
      c->op_scratch = nullptr;
      c->op_scratch_cap = 0;
    }
    if (hipMalloc(&c->op_scratch, bytes) != hipSuccess) {
      c->op_scratch = nullptr;
      (void)hipGetLastError();
      return fail(c, MG_ERR_OOM, "operator scratch allocation failed");
    }
    c->op_scratch_cap = bytes;
  }
  *out = reinterpret_cast<double*>(c->op_scratch);
  return MG_OK;
}

// `sweeps` full sweeps of u in place: on levels the streaming passes support, ping-ponging
// with the operator scratch (zero_in: u is zero on input and the first sweep does not read
// it, as in the first sweep of a mixed-precision correction cycle); else per colour.
template <typename T>
int op_smooth(mg_ctx* c, int n, double h, double omega, int sweeps, bool zero_in, const mg_level_bc* bc, T* u,
              const T* f, void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  if (n < 2 || sweeps < 0 || sweeps > 4) return fail(c, MG_ERR_INVALID_ARG, "n >= 2, sweeps 0..4");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const LevelBC b = to_level_bc(bc);
  if (fused_supported<T>(n) && sweeps > 0) {
    double* tmp = nullptr;
    st = op_scratch(c, cells(ilog2(n)) * sizeof(T), &tmp);
    if (st) return st;
    T* cur = u;
    T* oth = reinterpret_cast<T*>(tmp);
    for (int it = 0; it < sweeps; ++it) {
      fused_sweep<T>(it == 0 && zero_in ? nullptr : cur, oth, f, n, h, omega, b, s);
      std::swap(cur, oth);
    }
    if (cur != u) HIP_CHECK(c, hipMemcpyAsync(u, cur, cells(ilog2(n)) * sizeof(T), hipMemcpyDeviceToDevice, s));
  } else {
    if (zero_in && sweeps > 0) HIP_CHECK(c, hipMemsetAsync(u, 0, cells(ilog2(n)) * sizeof(T), s));
    for (int it = 0; it < sweeps; ++it)
      for (int colour = 0; colour < 2; ++colour) launch_half_sweep<T>(u, f, n, h, omega, colour, b, s);
  }
  return op_epilogue(c);
}

// Do the operator entry points run a V(2,2) leg of this level as one two-sweep streaming pass
// (the context's "march" setting, as in the solver; any level the passes support)?
template <typename T>
bool op_march(const mg_ctx* c, int n, int sweeps, const LevelBC& b) {
  const int v = c->march[sizeof(T) == 8 ? 0 : 1];
  const int mode = v < 0 ? 2 : v;
  if (mode == 0 || sweeps != 2 || n < kMarchMinN) return false;
  if (mode == 1)
    for (int f = 0; f < 6; ++f)
      if (b.kind[f] != BC_PERIODIC) return false;
  return true;
}

// The region-tile and streaming up passes take the coarse correction's ghosts from the face
// kinds alone (homogeneous conditions, no face values).
bool hom_arrays_null(const LevelBC& b) {
  for (int f = 0; f < 6; ++f)
    if (b.b[f]) return false;
  return true;
}

// Do the operator entry points run a V(2,2) leg of this level as one region-tile launch (the
// context's "tile" setting, on the levels the solver uses them for: 32^3 .. 128^3, below the
// streaming passes)?
template <typename T>
bool op_tile(const mg_ctx* c, int n, int sweeps) {
  const int v = c->tile[sizeof(T) == 8 ? 0 : 1];
  return (v < 0 || v == 1) && sweeps == 2 && n >= kTileMinN && n <= kTileMaxN && n < kFusedDefaultMinN;
}

// Down step (Alg. 1 steps 1-3) with the context's fusion schedule for this precision.
template <typename T>
int op_down(mg_ctx* c, int n, double h, double omega, int npre, const mg_level_bc* bc, T* u, const T* f, T* fc, T* uc,
            void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  if (n < 2 || npre < 0 || npre > 4) return fail(c, MG_ERR_INVALID_ARG, "n >= 2, npre 0..4");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const LevelBC b = to_level_bc(bc);
  if (op_march<T>(c, n, npre, b)) {
    double* tmp = nullptr;
    st = op_scratch(c, cells(ilog2(n)) * sizeof(T), &tmp);
    if (st) return st;
    march_down<T>(u, reinterpret_cast<T*>(tmp), f, fc, uc, n, h, omega, b, s);
    HIP_CHECK(c, hipMemcpyAsync(u, tmp, cells(ilog2(n)) * sizeof(T), hipMemcpyDeviceToDevice, s));
    return op_epilogue(c);
  }
  if (op_tile<T>(c, n, npre)) {
    double* tmp = nullptr;
    st = op_scratch(c, cells(ilog2(n)) * sizeof(T), &tmp);
    if (st) return st;
    tile_down<T>(u, reinterpret_cast<T*>(tmp), f, fc, uc, n, 0, 0, h, omega, b, s);
    HIP_CHECK(c, hipMemcpyAsync(u, tmp, cells(ilog2(n)) * sizeof(T), hipMemcpyDeviceToDevice, s));
    return op_epilogue(c);
  }
  if (fused_supported<T>(n) && npre > 0) {
    double* tmp = nullptr;
    st = op_scratch(c, cells(ilog2(n)) * sizeof(T), &tmp);
    if (st) return st;
    // the context's schedule, as in the solver: the restricted defect fused into the last
    // sweep or as its own pass
    auto it_split = c->pass_split.find((sizeof(T) == 8 ? 0 : 1000) + ilog2(n));
    const bool sdef = it_split != c->pass_split.end() ? (it_split->second & 1) != 0 : false;
    T* cur = u;
    T* oth = reinterpret_cast<T*>(tmp);
    for (int it = 0; it < npre; ++it) {
      if (it == npre - 1 && !sdef) fused_sweep_defect<T>(cur, oth, f, fc, uc, n, h, omega, b, s);
      else fused_sweep<T>(cur, oth, f, n, h, omega, b, s);
      std::swap(cur, oth);
    }
    if (sdef) fused_defect_restrict<T>(cur, f, fc, uc, n, h, b, s);
    if (cur != u) HIP_CHECK(c, hipMemcpyAsync(u, cur, cells(ilog2(n)) * sizeof(T), hipMemcpyDeviceToDevice, s));
    return op_epilogue(c);
  }
  st = op_smooth<T>(c, n, h, omega, npre, false, bc, u, f, stream);
  if (st) return st;
  launch_defect_restrict<T>(u, f, fc, uc, n, h, b, s);
  return op_epilogue(c);
}

// Up step (Alg. 1 steps 5-7): the prolonged correction enters with the first post-sweep.
template <typename T>
int op_up(mg_ctx* c, int n, double h, double omega, int npost, const mg_level_bc* bc, const mg_level_bc* bc_coarse,
          T* u, const T* f, const T* uc, void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  if (n < 2 || npost < 0 || npost > 4) return fail(c, MG_ERR_INVALID_ARG, "n >= 2, npost 0..4");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const LevelBC b = to_level_bc(bc), bcc = to_level_bc(bc_coarse);
  if (op_march<T>(c, n, npost, b) && hom_arrays_null(bcc)) {
    double* tmp = nullptr;
    st = op_scratch(c, cells(ilog2(n)) * sizeof(T), &tmp);
    if (st) return st;
    (void)march_up<T>(u, reinterpret_cast<T*>(tmp), f, uc, bcc, nullptr, n, h, omega, b, s);
    HIP_CHECK(c, hipMemcpyAsync(u, tmp, cells(ilog2(n)) * sizeof(T), hipMemcpyDeviceToDevice, s));
    return op_epilogue(c);
  }
  if (op_tile<T>(c, n, npost) && hom_arrays_null(bcc)) {
    double* tmp = nullptr;
    st = op_scratch(c, cells(ilog2(n)) * sizeof(T), &tmp);
    if (st) return st;
    (void)tile_up<T>(u, reinterpret_cast<T*>(tmp), f, uc, bcc, nullptr, n, 0, 0, h, omega, b, s);
    HIP_CHECK(c, hipMemcpyAsync(u, tmp, cells(ilog2(n)) * sizeof(T), hipMemcpyDeviceToDevice, s));
    return op_epilogue(c);
  }
  if (fused_supported<T>(n) && npost > 0) {
    double* tmp = nullptr;
    st = op_scratch(c, cells(ilog2(n)) * sizeof(T), &tmp);
    if (st) return st;
    T* cur = u;
    T* oth = reinterpret_cast<T*>(tmp);
    for (int it = 0; it < npost; ++it) {
      if (it == 0) fused_prolong_sweep<T>(cur, oth, f, uc, bcc, n, h, omega, b, s);
      else fused_sweep<T>(cur, oth, f, n, h, omega, b, s);
      std::swap(cur, oth);
    }
    if (cur != u) HIP_CHECK(c, hipMemcpyAsync(u, cur, cells(ilog2(n)) * sizeof(T), hipMemcpyDeviceToDevice, s));
    return op_epilogue(c);
  }
  launch_prolong<T>(uc, u, n / 2, bcc, 0, s);
  return op_smooth<T>(c, n, h, omega, npost, false, bc, u, f, stream);
}

}  // namespace

extern "C" {

int mg_op_half_sweep(mg_ctx* c, int n, double h, double omega, int colour, const mg_level_bc* bc, double* u,
                     const double* f, void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  if (n < 2 || (colour != 0 && colour != 1)) return fail(c, MG_ERR_INVALID_ARG, "n >= 2, colour 0 or 1");
  launch_half_sweep<double>(u, f, n, h, omega, colour, to_level_bc(bc), reinterpret_cast<hipStream_t>(stream));
  return op_epilogue(c);
}

int mg_op_smooth(mg_ctx* c, int n, double h, double omega, int sweeps, const mg_level_bc* bc, double* u,
                 const double* f, void* stream) {
  return op_smooth<double>(c, n, h, omega, sweeps, false, bc, u, f, stream);
}

int mg_op_smooth_f32(mg_ctx* c, int n, double h, double omega, int sweeps, int zero_in, const mg_level_bc* bc,
                     float* u, const float* f, void* stream) {
  return op_smooth<float>(c, n, h, omega, sweeps, zero_in != 0, bc, u, f, stream);
}

int mg_op_fill(mg_ctx* c, int n, const mg_level_bc* bc, const double* u, double* out, void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  if (!u || !out) return fail(c, MG_ERR_INVALID_ARG, "null u or out");
  launch_fill(u, out, n, to_level_bc(bc), reinterpret_cast<hipStream_t>(stream));
  return op_epilogue(c);
}

int mg_op_defect(mg_ctx* c, int n, double h, const mg_level_bc* bc, const double* u, const double* f, double* d,
                 void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  launch_defect<double>(u, f, d, n, h, to_level_bc(bc), reinterpret_cast<hipStream_t>(stream));
  return op_epilogue(c);
}

int mg_op_restrict(mg_ctx* c, int nc, const double* uf, double* uc, void* stream) {
  int st = op_prologue(c, nc);
  if (st) return st;
  launch_restrict<double, double>(uf, uc, nc, reinterpret_cast<hipStream_t>(stream));
  return op_epilogue(c);
}

int mg_op_prolong_add(mg_ctx* c, int nc, const mg_level_bc* bc, const double* uc, double* uf, void* stream) {
  int st = op_prologue(c, nc);
  if (st) return st;
  launch_prolong<double>(uc, uf, nc, to_level_bc(bc), 0, reinterpret_cast<hipStream_t>(stream));
  return op_epilogue(c);
}

int mg_op_prolong_fmg(mg_ctx* c, int nc, const mg_level_bc* bc, const double* uc, double* uf, void* stream) {
  int st = op_prologue(c, nc);
  if (st) return st;
  launch_prolong<double>(uc, uf, nc, to_level_bc(bc), 1, reinterpret_cast<hipStream_t>(stream));
  return op_epilogue(c);
}

int mg_op_coarsest(mg_ctx* c, double h, const mg_level_bc* bc, double* u, const double* f, void* stream) {
  int st = op_prologue(c, 1);
  if (st) return st;
  launch_coarsest<double>(u, f, h, to_level_bc(bc), reinterpret_cast<hipStream_t>(stream));
  return op_epilogue(c);
}

int mg_op_down(mg_ctx* c, int n, double h, double omega, int npre, const mg_level_bc* bc, double* u, const double* f,
               double* fc, double* uc, void* stream) {
  return op_down<double>(c, n, h, omega, npre, bc, u, f, fc, uc, stream);
}

int mg_op_down_f32(mg_ctx* c, int n, double h, double omega, int npre, const mg_level_bc* bc, float* u, const float* f,
                   float* fc, float* uc, void* stream) {
  return op_down<float>(c, n, h, omega, npre, bc, u, f, fc, uc, stream);
}

int mg_op_up(mg_ctx* c, int n, double h, double omega, int npost, const mg_level_bc* bc, const mg_level_bc* bc_coarse,
             double* u, const double* f, const double* uc, void* stream) {
  return op_up<double>(c, n, h, omega, npost, bc, bc_coarse, u, f, uc, stream);
}

int mg_op_up_f32(mg_ctx* c, int n, double h, double omega, int npost, const mg_level_bc* bc,
                 const mg_level_bc* bc_coarse, float* u, const float* f, const float* uc, void* stream) {
  return op_up<float>(c, n, h, omega, npost, bc, bc_coarse, u, f, uc, stream);
}

int mg_op_sweep_input_norm(mg_ctx* c, int n, double h, double omega, const mg_level_bc* bc, double* u,
                           const double* f, double* sumsq, void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  if (n < 2 || !u || !f || !sumsq) return fail(c, MG_ERR_INVALID_ARG, "n >= 2 and every array");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const LevelBC b = to_level_bc(bc);
  const size_t n3 = cells(ilog2(n));
  if (fused_supported<double>(n)) {
    // the solver's head pass: the sweep, with the defect of its input summed on the way
    double* tmp = nullptr;
    st = op_scratch(c, n3 * sizeof(double), &tmp);
    if (st) return st;
    const int np = fused_sweep_input_norm<double>(u, tmp, f, c->part, n, h, omega, b, s);
    launch_sum_partials(c->part, np, c->scal + 2, s);
    HIP_CHECK(c, hipMemcpyAsync(u, tmp, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    launch_defect_norm(u, f, nullptr, n, h, b, c->part, c->scal + 2, s);
    for (int colour = 0; colour < 2; ++colour) launch_half_sweep<double>(u, f, n, h, omega, colour, b, s);
  }
  HIP_CHECK(c, hipMemcpyAsync(c->hscal + 2, c->scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_CHECK(c, hipStreamSynchronize(s));
  *sumsq = c->hscal[2];
  return op_epilogue(c);
}

int mg_op_mixed_update(mg_ctx* c, int n, double h, const mg_level_bc* bc, double* phi, const float* e, const double* f,
                       float* r32, double* sumsq, void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  if (n < 2 || !phi || !e || !f || !r32 || !sumsq) return fail(c, MG_ERR_INVALID_ARG, "n >= 2 and every array");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const LevelBC b = to_level_bc(bc);
  const size_t n3 = cells(ilog2(n));
  if (n >= kFusedMinN) {
    // the solver's streaming pass: phi + e, its defect, the FP32 copy and the partial sums
    double* tmp = nullptr;
    st = op_scratch(c, n3 * sizeof(double), &tmp);
    if (st) return st;
    const int np = fused_mixed_update_defect(phi, tmp, e, f, r32, c->part, n, h, b, s);
    launch_sum_partials(c->part, np, c->scal + 2, s);
    HIP_CHECK(c, hipMemcpyAsync(phi, tmp, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    launch_add_f32(phi, e, n3, s);
    launch_defect_norm(phi, f, r32, n, h, b, c->part, c->scal + 2, s);
  }
  HIP_CHECK(c, hipMemcpyAsync(c->hscal + 2, c->scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_CHECK(c, hipStreamSynchronize(s));
  *sumsq = c->hscal[2];
  return op_epilogue(c);
}

int mg_multipole_moments(mg_ctx* c, int n, double dx, const double* rho, int lmax, int use_origin, const double* origin,
                         double* origin_out, double* q_out, void* stream) {
  int st = op_prologue(c, n);
  if (st) return st;
  if (lmax < 0 || lmax > 4) return fail(c, MG_ERR_INVALID_ARG, "lmax in 0..4");
  if (use_origin && !origin) return fail(c, MG_ERR_INVALID_ARG, "origin required");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* mps = c->scal + kMpoleOff;
  HIP_CHECK(c, hipMemsetAsync(c->scal, 0, sizeof(double) * kScal, s));
  launch_multipole_moments(rho, n, 0, dx, lmax, use_origin, origin, c->part, mps, s);
  HIP_CHECK(c, hipMemcpyAsync(c->hscal, c->scal, sizeof(double) * kScal, hipMemcpyDeviceToHost, s));
  HIP_CHECK(c, hipStreamSynchronize(s));
  if (origin_out)
    for (int a = 0; a < 3; ++a) origin_out[a] = c->hscal[kMpoleOff + 4 + a];
  if (q_out)
    for (int q = 0; q < 25; ++q) q_out[q] = c->hscal[kMpoleOff + 7 + q];
  return op_epilogue(c);
}

int mg_amr_solve(mg_ctx* c, const mg_params* p, const mg_amr_mesh* mesh, const mg_bc* bc, const double* const* rho,
                 double* const* phi, double* hist, int* n_hist, void* stream) {
  if (!c) return MG_ERR_INVALID_ARG;
  if (n_hist) *n_hist = 0;
  std::vector<double> hpart((size_t)kMaxPartials * (MG_AMR_MAX_LEVELS + 1));   // one row of partials per patch
  // what the budget leaves for the refined-mesh workspace (its current size included)
  size_t room = SIZE_MAX;
  if (c->hbm_budget) {
    const size_t other = kFixedBytes + c->ws_cap + c->op_scratch_cap;
    room = c->hbm_budget > other ? c->hbm_budget - other : 0;
  }
  return amr_solve_impl(c->device, p, mesh, bc, rho, phi, hist, n_hist, stream, c->part, hpart.data(), &c->amr_ws,
                        &c->amr_ws_cap, room, &c->err);
}

int mg_gravity(mg_ctx* c, const mg_params* p, const mg_bc* bc, const double* phi, const double* rho, double* g,
               double* rhog, double* gface, void* stream) {
  if (!c) return MG_ERR_INVALID_ARG;
  int st = validate(c, p, bc);
  if (st != MG_OK) return st;
  if (!phi) return fail(c, MG_ERR_INVALID_ARG, "null phi");
  if (!g && !rhog && !gface) return fail(c, MG_ERR_INVALID_ARG, "no output requested");
  bool any_mp = false, any_fixed = false;
  for (int f = 0; f < 6; ++f) {
    any_mp |= bc->kind[f] == MG_BC_MULTIPOLE;
    any_fixed |= bc->kind[f] == MG_BC_FIXED && bc->fixed_b[f];
  }
  if ((rhog || any_mp) && !rho) return fail(c, MG_ERR_INVALID_ARG, "rho is required for rhog and multipole faces");
  const int Lb = layout_lb(p);
  if (gface && Lb >= 0) return fail(c, MG_ERR_UNSUPPORTED, "face accelerations are written for the dense layout only");
  HIP_CHECK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int n = p->n, L = ilog2(n);
  const int Lm = Lb >= 0 ? L - Lb : 0;
  // boundary description of the finest level, as the solve builds it (Sec. 2.3.6, App. A)
  LevelBC lb;
  double* fb = nullptr;
  if (any_mp || any_fixed) {
    st = op_scratch(c, 6 * face_sz(L) * sizeof(double), &fb);
    if (st) return st;
  }
  double* mp_out[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int f = 0; f < 6; ++f) {
    const int k = bc->kind[f];
    lb.kind[f] = k == MG_BC_MULTIPOLE ? MG_BC_FIXED : k;
    lb.b[f] = nullptr;
    double* e = fb ? fb + (size_t)f * face_sz(L) : nullptr;
    if (k == MG_BC_FIXED && bc->fixed_b[f]) {
      launch_face_extend(bc->fixed_b[f], e, n, s);
      lb.b[f] = e;
    } else if (k == MG_BC_MULTIPOLE) {
      mp_out[f] = e;
      lb.b[f] = e;
    }
  }
  if (any_mp) {
    double* mps = c->scal + kMpoleOff;
    launch_multipole_moments(rho, n, Lm, p->dx, bc->lmax, bc->use_origin, bc->origin, c->part, mps, s);
    launch_multipole_faces(mps, bc->lmax, p->four_pi_g / (4.0 * M_PI), n, p->dx, n * p->dx, mp_out, s);
  }
  launch_gravity(phi, rho, g, rhog, gface, n, Lm, p->dx, lb, s);
  return op_epilogue(c);
}

int mg_gravity_kernel_name(const mg_params* p, int want_g, int want_rhog, int want_gface, char* buf, int cap) {
  if (!p || !is_pow2(p->n) || p->n < 2) return MG_ERR_INVALID_ARG;
  const int Lb = layout_lb(p);
  const std::string nm =
      gravity_kernel_name(p->n, Lb >= 0 ? ilog2(p->n) - Lb : 0, want_g != 0, want_rhog != 0, want_gface != 0);
  const int len = (int)nm.size() + 1;
  if (buf && cap > 0) {
    std::strncpy(buf, nm.c_str(), (size_t)cap);
    buf[cap - 1] = 0;
  }
  return len;
}

}  // extern "C"

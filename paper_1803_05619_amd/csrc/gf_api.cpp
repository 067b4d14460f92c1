// C ABI of the guided filtering layer: argument checks, launch planning,
// workspace layout and kernel timing.  Every check runs on the host before
// any HIP call, so invalid input is reported without touching a device.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "gf_internal.h"

namespace gf {
namespace {

thread_local std::string g_detail;

int fail(int code, const std::string& why) {
  g_detail = why;
  return code;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int dtype_size(int t) {
  switch (t) {
    case GF_F32: return 4;
    case GF_F16: return 2;
    case GF_BF16: return 2;
  }
  return 0;
}

// Largest radius the column-walker kernels take: a wave of 64 lanes covers
// the output columns plus a halo of 2r on each side.
constexpr int kMaxRadius = 10;

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v ? atoi(v) : dflt;
}

}  // namespace

int wide_coef_min_r() {
  static const int v = std::max(kWideMinR, env_int("GF_WIDE_COEF_R", kWideCoefR));
  return v;
}
int wide_bwd_min_r() {
  static const int v = std::max(kWideMinR, env_int("GF_WIDE_BWD_R", kWideBwdR));
  return v;
}

int set_error(int code, const std::string& why) { return fail(code, why); }

int make_plan(const gf_desc_t* d, const gf_guide_t* g, Plan* p, const char** why) {
  static thread_local std::string msg;
  auto bad = [&](int code, const std::string& m) {
    msg = m;
    *why = msg.c_str();
    return code;
  };
  if (!d) return bad(GF_ERR_INVALID_ARG, "desc is NULL");
  if (d->n < 1 || d->c < 1) return bad(GF_ERR_INVALID_ARG, "n and c must be >= 1");
  if (d->h_lo < 1 || d->w_lo < 1 || d->h_hi < 1 || d->w_hi < 1)
    return bad(GF_ERR_INVALID_ARG, "image sizes must be >= 1");
  if (d->h_lo > d->h_hi || d->w_lo > d->w_hi)
    return bad(GF_ERR_INVALID_ARG, "low-res size must not exceed high-res size");
  if (d->r < 0) return bad(GF_ERR_INVALID_ARG, "radius r must be >= 0");
  if (d->mean_ab != 0 && d->mean_ab != 1) return bad(GF_ERR_INVALID_ARG, "mean_ab must be 0 or 1");
  if (d->align_corners != 0 && d->align_corners != 1)
    return bad(GF_ERR_INVALID_ARG, "align_corners must be 0 or 1");
  if (d->precise != 0 && d->precise != 1) return bad(GF_ERR_INVALID_ARG, "precise must be 0 or 1");
  if (dtype_size(d->io_dtype) == 0) return bad(GF_ERR_INVALID_ARG, "unknown io_dtype");
  // one integer factor in {1, 2, 4, 8} for both axes takes the kernels with
  // compile-time tap weights; any other ratio (per axis) the general ones
  int S = 0;
  if (d->h_hi % d->h_lo == 0 && d->w_hi % d->w_lo == 0 &&
      d->h_hi / d->h_lo == d->w_hi / d->w_lo) {
    S = d->h_hi / d->h_lo;
    if (S != 1 && S != 2 && S != 4 && S != 8) S = 0;
  }
  const double hi_elems = (double)d->n * d->c * d->h_hi * d->w_hi;
  if (hi_elems > 9.0e15 || (double)d->h_hi * d->w_hi > 2.0e9)
    return bad(GF_ERR_UNSUPPORTED, "problem too large");
  const int gmode = g ? g->mode : GF_GUIDE_IDENTITY;
  if (gmode != GF_GUIDE_IDENTITY && gmode != GF_GUIDE_GREY && gmode != GF_GUIDE_TRANSFORM)
    return bad(GF_ERR_INVALID_ARG, "unknown guide mode");
  const int c_in = gmode == GF_GUIDE_IDENTITY ? d->c : g->c_in;
  if (gmode == GF_GUIDE_IDENTITY && g && g->c_in != 0 && g->c_in != d->c)
    return bad(GF_ERR_INVALID_ARG, "identity guide needs c_in == c");
  if (gmode == GF_GUIDE_GREY && (c_in < 1 || c_in > 4 || d->c > 4))
    return bad(GF_ERR_UNSUPPORTED, "grey guide supports 1..4 input and output channels");
  if (gmode == GF_GUIDE_TRANSFORM) {
    if (c_in != 3 || d->c != 3) return bad(GF_ERR_UNSUPPORTED, "transform guide needs c_in == c == 3");
    if (g->hidden < 1 || g->hidden > 16) return bad(GF_ERR_UNSUPPORTED, "transform hidden width must be 1..16");
    if (!g->params) return bad(GF_ERR_INVALID_ARG, "transform guide needs params");
    if (!(g->bn_eps >= 0.f)) return bad(GF_ERR_INVALID_ARG, "bn_eps must be >= 0");
    if (g->use_stats && !g->stats) return bad(GF_ERR_INVALID_ARG, "use_stats needs stats");
  }
  Plan& q = *p;
  q.gmode = gmode;
  q.c_in = c_in;
  q.hidden = gmode == GF_GUIDE_TRANSFORM ? g->hidden : 0;
  q.KP = 16;
  q.bn_eps = g ? g->bn_eps : 0.f;
  q.slope = g ? g->slope : 0.f;
  q.gparams = g ? g->params : nullptr;
  q.gstats = g ? g->stats : nullptr;
  q.use_stats = g ? g->use_stats : 0;
  q.n = d->n;
  q.c = d->c;
  q.h = d->h_lo;
  q.w = d->w_lo;
  q.H = d->h_hi;
  q.W = d->w_hi;
  q.r = d->r;
  q.mean_ab = d->mean_ab;
  q.ac = d->align_corners;
  q.wide_co = wide_coef(d->r) || d->precise;
  q.wide_lo = wide_bwd(d->r) || d->precise;
  q.dtype = d->io_dtype;
  q.S = S;
  q.gen = S == 0;
  q.xcd = std::max(0, env_int("GF_XCD", 0));  // workgroup order run; see xcd_order
  // the low-res walkers' strips in XCD-contiguous runs (neighbouring strips
  // share halo cache lines): on the FP32 4 x 3 x 2048 x 3072 step the
  // coefficients 24.1 -> 20.8 us and the low-res backward 43.0 -> 35.3 us;
  // neutral on the FP16 2 x 3 x 2160 x 3840 step
  q.lo_xcd = std::max(0, env_int("GF_LO_XCD", 1));
  q.planes = d->n * d->c;
  // elements per lane-load on the high-res side: 4 (16 bytes of float, 8 of
  // a half type), 1 when W is not a multiple
  int V = 4;
  q.VEC = (q.W % V == 0) ? V : 1;

  const int r = q.r;
  if (r > kMaxRadius) return bad(GF_ERR_UNSUPPORTED, "radius above 10 is not supported");
  const int hal = q.mean_ab ? 2 * r : r;  // halo of the coefficient walker
  // Launch shapes: the tuned entry for this key if the autotuner (or an
  // import) made one, else the defaults below; environment overrides win
  // (tuning experiments).
  //  - rows per low-res walker wave: 16 (coefficients) / 24 (backward) for
  //    r <= 2 (enough waves to fill the chip in one round; the register
  //    windows make the 2*halo warm-up rows cheap), longer for larger radii
  //    to amortise their warm-up
  //  - high-res rows per apply thread: short walks keep DRAM streams
  //    sequential (8 measured best on MI355X for the 4 x 3 x 2048 x 3072
  //    workload): two low-res row blocks at S = 4, one at S = 8
  //  - low-res rows per backward high-res wave: 2 for FP32 (short walks
  //    stream best; at S >= 4 four waves stack into one partial block), 8
  //    for the half types (one wave per workgroup: fewer partial rows)
  //  - the wide passes (large r): see one_round below
  const int walk = r <= 2 ? 16 : r <= 4 ? 32 : 64;
  // the backward walker at small radii: 24 rows (4 waves per SIMD; 16-row
  // segments leave a second, mostly empty round of waves)
  TuneVal tv{walk, r <= 2 ? 24 : r <= 4 ? walk : 128, S >= 8 ? S : 8,
             d->io_dtype == GF_F32 ? 2 : 8};
  TuneVal tuned;
  const bool tuned_hit = tune_lookup(TuneKey{d->io_dtype, S, r, gmode, d->mean_ab}, &tuned);
  if (tuned_hit) {
    tv = tuned;
  } else if (r <= 2) {
    // small problems (latency-bound launches): shorter walks spread the
    // low-res walkers and the apply threads over more of the chip, down to
    // 4 rows (a quarter of the default) while fewer than 1024 waves or 256
    // apply workgroups would run
    const long long planes = (long long)d->n * d->c;
    const int hal_c = d->mean_ab ? 2 * r : r;
    const long long nx_c = (d->w_lo + (64 - 2 * hal_c) - 1) / (64 - 2 * hal_c);
    const long long nx_l = (d->w_lo + (64 - 4 * r) - 1) / (64 - 4 * r);
    auto waves = [&](long long nx, int tr) { return nx * ((d->h_lo + tr - 1) / tr) * planes; };
    while (tv.coTR > 4 && waves(nx_c, tv.coTR) < 1024) tv.coTR /= 2;
    while (tv.loTR > 6 && waves(nx_l, tv.loTR) < 1024) tv.loTR /= 2;
    const long long vec = d->w_hi % 4 == 0 ? 4 : 1;
    auto apply_wgs = [&](int rb) {
      return planes * ((d->h_hi + rb - 1) / rb) * (d->w_hi / vec) / 256;
    };
    while (tv.RB > std::max(S, 1) && apply_wgs(tv.RB) < 256) tv.RB /= 2;
  }
  // the wide passes (when nothing was tuned): the row tile that fills one
  // round of resident workgroups (LDS-limited: 3 per CU for the coefficient
  // passes, 2 for the backward's), multiples of 8 from 16 rows; a problem too
  // large for one round at 128 rows takes 64 (its halo rows then matter
  // more than the tail of the last round).  Measured at r = 8 on the FP16
  // 2 x 3 x 2160 x 3840 workload, the backward's two passes: 125 / 145 /
  // 106 / 135 us at 16 / 24 / 32 / 48 rows (408 workgroups at 32 rows fit
  // the 512 resident, 552 at 24 do not).
  auto one_round = [&](int cap_per_cu, int nx) {
    const long long planes = (long long)d->n * d->c;
    for (int tr = 16; tr <= 128; tr += 8)
      if (nx * planes * ((d->h_lo + tr - 1) / tr) <= 256LL * cap_per_cu) return tr;
    return 64;
  };
  if (!tuned_hit) {
    const int nxw = (d->w_lo + (kWideBThreads - 2 * r) - 1) / (kWideBThreads - 2 * r);
    if (q.wide_co) tv.coTR = one_round((int)(kLdsPerCU / wide_lds_bytes(4)), nxw);
    if (q.wide_lo) tv.loTR = one_round((int)(kLdsPerCU / wide_lds_bytes(6)), nxw);
  }
  if (env_int("GF_LO_ROWS", 0) > 0) tv.coTR = tv.loTR = env_int("GF_LO_ROWS", 0);
  if (env_int("GF_BWD_LO_ROWS", 0) > 0) tv.loTR = env_int("GF_BWD_LO_ROWS", 0);
  if (env_int("GF_APPLY_ROWS", 0) > 0) tv.RB = env_int("GF_APPLY_ROWS", 0);
  if (env_int("GF_BWD_BH", 0) >= 2) tv.bh = env_int("GF_BWD_BH", 0);
  if (tv.coTR < 1 || tv.loTR < 1 || tv.RB < 1 || tv.bh < 2)
    return bad(GF_ERR_INVALID_ARG, "invalid launch shape");
  q.coTR = tv.coTR;
  if (q.wide_co) {  // wide coefficient passes: strips of 256 input columns, halo r
    q.co_nx = (q.w + (kWideBThreads - 2 * r) - 1) / (kWideBThreads - 2 * r);
    q.coLDS = bwd_wide_lds_bytes();
  } else {
    q.co_nx = (q.w + (64 - 2 * hal) - 1) / (64 - 2 * hal);
    q.coLDS = coef_lds_bytes(r);  // row buffers (+ (g,p), (A,b) rings for large r)
  }
  q.co_ny = (q.h + q.coTR - 1) / q.coTR;
  q.loTR = tv.loTR;
  if (q.wide_lo) {  // wide backward: strips of 256 input columns, halo r
    q.lo_nx = (q.w + (kWideBThreads - 2 * r) - 1) / (kWideBThreads - 2 * r);
    q.loLDS = bwd_wide_lds_bytes();
  } else {
    q.lo_nx = (q.w + (64 - 4 * r) - 1) / (64 - 4 * r);
    q.loLDS = bwd_lo_lds_bytes(r);  // row buffers (+ input and X rings for large r)
  }
  q.lo_ny = (q.h + q.loTR - 1) / q.loTR;

  q.RB = S ? ((tv.RB + S - 1) / S) * S : tv.RB;  // whole low-res row blocks
  q.nrb = (q.H + q.RB - 1) / q.RB;
  q.nxv = q.W / q.VEC;

  if (S) {
    q.tw = 64 * q.VEC / S;
    q.hw = hi_merge(d->io_dtype == GF_F32, S) ? kHiWaves : 1;  // waves per high-res workgroup
    q.bh = tv.bh;  // rows per wave; fewer when the workgroup's merge buffers would exceed 64 KB
    while (q.bh > 2 && bwd_hi_lds_bytes(q.hw * q.bh, q.tw) > kHiLdsMax) --q.bh;
    q.ubh = q.hw * q.bh;
    q.hiLDS = bwd_hi_lds_bytes(q.ubh, q.tw);
    q.nby = (q.h + q.ubh - 1) / q.ubh;
    q.nbx = (q.W + 64 * q.VEC - 1) / (64 * q.VEC);
  } else {
    // any ratio: the partial planes are one block per plane, the whole
    // low-res plane with a border of one row and column
    q.tw = q.w;
    q.hw = 1;
    q.bh = q.ubh = q.h;
    q.hiLDS = 0;
    q.nby = q.nbx = 1;
  }
  q.ublk_floats = (size_t)2 * (q.ubh + 2) * (q.tw + 2);
  // the low-res walkers address a plane, and its partial planes, with
  // 32-bit byte offsets
  if ((double)q.h * q.w * 4.0 > 2147483647.0 ||
      (double)q.nby * q.nbx * q.ublk_floats * 4.0 > 2147483647.0)
    return bad(GF_ERR_UNSUPPORTED, "low-res plane too large");

  const size_t lo_plane = (size_t)q.planes * q.h * q.w * sizeof(float);
  q.off_abar = 0;
  q.off_bbar = align_up(lo_plane, 256);
  q.ws_fwd = q.off_bbar + align_up(lo_plane, 256);
  // the partial planes follow bbar (not aliasing it: the fused forward +
  // backward pass reads bbar while it writes them)
  q.off_u = q.off_bbar + align_up(lo_plane, 256);
  const size_t ubytes = (size_t)q.planes * q.nby * q.nbx * q.ublk_floats * sizeof(float);
  q.off_v = q.off_u + align_up(ubytes, 256);
  const size_t vbytes = q.gen ? (size_t)q.planes * 2 * q.h * q.W * sizeof(float) : 0;
  q.off_eps = q.off_v + align_up(vbytes, 256);
  q.off_x = q.off_eps + align_up((size_t)q.planes * q.lo_nx * q.lo_ny * sizeof(float), 256);
  // the wide passes' plane: X of the backward (16 bytes per pixel, 32 in
  // FP64 for FP32 I/O), or the coefficients' (A, b) (8), which the
  // forward-only calls need as well
  const bool wide_x = q.wide_lo || (q.wide_co && q.mean_ab);
  const size_t xbytes = wide_x ? (size_t)q.planes * q.h * q.w * wide_x_floats(q) * sizeof(float) : 0;
  q.ws_bwd = q.off_x + align_up(xbytes, 256);
  if (q.wide_co && q.mean_ab) q.ws_fwd = std::max(q.ws_fwd, q.ws_bwd);
  if (gmode != GF_GUIDE_IDENTITY) {
    // guided path: the guide planes and the transform's reductions follow the
    // identity layout (a superset is allocated for both directions)
    const size_t lo = (size_t)q.planes * q.h * q.w * sizeof(float);
    const size_t hi = (size_t)q.planes * q.H * q.W * sizeof(float);
    // reduction chunks per image: about 8 K pixels each (enough workgroups
    // to fill the chip), at most 256
    auto chunks = [](long long P) { return (int)std::min<long long>(256, (P + 8191) / 8192); };
    q.g_chunks_lo = chunks((long long)q.h * q.w);
    q.g_chunks_hi = chunks((long long)q.H * q.W);
    size_t o = align_up(std::max(q.ws_fwd, q.ws_bwd), 256);
    q.off_gl = o;
    o += align_up(lo, 256);
    q.off_gh = o;
    o += align_up(hi, 256);
    q.ws_fwd = o;  // forward: G_l, G_h (+ the shared statistics below)
    q.off_dgl = o;
    o += align_up(lo, 256);
    q.off_dgh = o;
    o += align_up(hi, 256);
    q.off_mom = o;
    o += align_up(sizeof(float) * kMomFloats * q.n * std::max(q.g_chunks_lo, q.g_chunks_hi) * 2, 256);
    q.off_fold = o;
    o += align_up(sizeof(float) * kFoldFloats * 2, 256);
    q.off_accp = o;
    o += align_up(sizeof(float) * kAccFloats * q.n * std::max(q.g_chunks_lo, q.g_chunks_hi) * 2, 256);
    q.off_acct = o;
    o += align_up(sizeof(float) * kAccFloats * 2, 256);
    q.off_mlo = o;
    o += align_up(sizeof(uint16_t) * q.n * q.h * q.w, 256);
    q.off_mhi = o;
    o += align_up(sizeof(uint16_t) * q.n * q.H * q.W, 256);
    q.ws_bwd = o;
    // the forward also needs the moments and folded parameters: place them
    // after G_h as well (same offsets as in the backward layout are not
    // required, the forward uses only its own)
    q.ws_fwd = q.ws_bwd;
  }
  return GF_OK;
}

namespace {
hipError_t launch_forward(const Plan& p, const FwdArgs& a, hipStream_t s) {
  if (p.gmode != GF_GUIDE_IDENTITY) {
    switch (p.dtype) {
      case GF_F32: return launch_forward_guided_f32(p, a, s);
      case GF_F16: return launch_forward_guided_f16(p, a, s);
      case GF_BF16: return launch_forward_guided_bf16(p, a, s);
    }
    return hipErrorInvalidValue;
  }
  switch (p.dtype) {
    case GF_F32: return launch_forward_f32(p, a, s);
    case GF_F16: return launch_forward_f16(p, a, s);
    case GF_BF16: return launch_forward_bf16(p, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_backward(const Plan& p, const BwdArgs& a, hipStream_t s) {
  if (p.gmode != GF_GUIDE_IDENTITY) {
    switch (p.dtype) {
      case GF_F32: return launch_backward_guided_f32(p, a, s);
      case GF_F16: return launch_backward_guided_f16(p, a, s);
      case GF_BF16: return launch_backward_guided_bf16(p, a, s);
    }
    return hipErrorInvalidValue;
  }
  switch (p.dtype) {
    case GF_F32: return launch_backward_f32(p, a, s);
    case GF_F16: return launch_backward_f16(p, a, s);
    case GF_BF16: return launch_backward_bf16(p, a, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace

// ------------------------------------------------------------ profiling

namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<Rec> g_recs;
const char* g_pending_name = nullptr;
hipEvent_t g_pending_ev = nullptr;

// Recorded events go back to a pool (creating events costs far more host
// time than recording them, and the records sit in the timed region).
std::vector<hipEvent_t> g_ev_pool;

hipEvent_t ev_get() {
  if (!g_ev_pool.empty()) {
    hipEvent_t e = g_ev_pool.back();
    g_ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void prof_clear() {
  for (auto& r : g_recs) {
    g_ev_pool.push_back(r.a);
    g_ev_pool.push_back(r.b);
  }
  g_recs.clear();
  if (g_pending_ev) g_ev_pool.push_back(g_pending_ev);
  g_pending_ev = nullptr;
}
}  // namespace

thread_local bool g_prof_muted = false;
void prof_mute(bool on) { g_prof_muted = on; }

void prof_begin(const char* name, hipStream_t s) {
  if (g_prof_muted) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  hipEvent_t ev = ev_get();
  if (!ev) return;
  (void)hipEventRecord(ev, s);
  g_pending_name = name;
  g_pending_ev = ev;
}

void prof_end(hipStream_t s) {
  if (g_prof_muted) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on || !g_pending_ev) return;
  hipEvent_t ev = ev_get();
  if (!ev) return;
  (void)hipEventRecord(ev, s);
  g_recs.push_back({g_pending_name, g_pending_ev, ev});
  g_pending_ev = nullptr;
}

}  // namespace gf

// ------------------------------------------------------------ C ABI

using gf::fail;

static bool misaligned(const void* ptr) { return ((uintptr_t)ptr & 15u) != 0; }

extern "C" {

size_t gf_guide_param_count(int32_t c_in, int32_t c, int32_t hidden) {
  if (c_in < 1 || c < 1 || hidden < 1) return 0;
  return (size_t)hidden * c_in + (size_t)c * hidden + c + 2 + 2 * (size_t)hidden;
}

size_t gf_guide_stats_count(int32_t c_in) {
  if (c_in < 1) return 0;
  return 2 * ((size_t)c_in + (size_t)c_in * c_in);
}

size_t gf_workspace_size(const gf_desc_t* desc, const gf_guide_t* guide, int32_t backward) {
  gf::Plan p;
  const char* why = nullptr;
  if (gf::make_plan(desc, guide, &p, &why) != GF_OK) return 0;
  if (backward == 2) return std::max(p.ws_fwd, p.ws_bwd);
  return backward ? p.ws_bwd : p.ws_fwd;
}

int32_t gf_forward(const gf_desc_t* desc, const gf_guide_t* guide, const void* I_lo,
                   const void* p_lo, const void* I_hi, const float* eps, int32_t eps_count,
                   void* q_hi, void* ws, size_t ws_bytes, void* stream) {
  gf::g_detail.clear();
  gf::Plan p;
  const char* why = nullptr;
  int st = gf::make_plan(desc, guide, &p, &why);
  if (st != GF_OK) return fail(st, why);
  if (!I_lo || !p_lo || !I_hi || !eps || !q_hi)
    return fail(GF_ERR_INVALID_ARG, "a required pointer is NULL");
  if (eps_count != 1 && eps_count != desc->n)
    return fail(GF_ERR_INVALID_ARG, "eps_count must be 1 or n");
  if (misaligned(I_lo) || misaligned(p_lo) || misaligned(I_hi) || misaligned(q_hi) ||
      misaligned(ws))
    return fail(GF_ERR_INVALID_ARG, "tensor pointers must be 16-byte aligned");
  if (!ws || ws_bytes < p.ws_fwd)
    return fail(GF_ERR_WORKSPACE, "workspace smaller than gf_workspace_size(desc, guide, 0) = " +
                                      std::to_string(p.ws_fwd));
  gf::FwdArgs a{I_lo, p_lo, I_hi, eps, eps_count, q_hi, static_cast<char*>(ws)};
  hipError_t e = gf::launch_forward(p, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(GF_ERR_HIP, hipGetErrorString(e));
  return GF_OK;
}

}  // extern "C"

namespace {
// gf_backward, and with q_hi set gf_forward_backward.
int32_t run_backward(const gf_desc_t* desc, const gf_guide_t* guide, const void* I_lo,
                     const void* p_lo, const void* I_hi, const float* eps, int32_t eps_count,
                     const void* dq_hi, void* q_hi, float* dI_lo, float* dp_lo, void* dI_hi,
                     float* deps, float* dparams, void* ws, size_t ws_bytes, void* stream,
                     bool with_forward) {
  gf::g_detail.clear();
  gf::Plan p;
  const char* why = nullptr;
  int st = gf::make_plan(desc, guide, &p, &why);
  if (st != GF_OK) return fail(st, why);
  if (!I_lo || !p_lo || !I_hi || !eps || !dq_hi || (with_forward && !q_hi))
    return fail(GF_ERR_INVALID_ARG, "a required pointer is NULL");
  if (eps_count != 1 && eps_count != desc->n)
    return fail(GF_ERR_INVALID_ARG, "eps_count must be 1 or n");
  if (dparams && p.gmode != GF_GUIDE_TRANSFORM)
    return fail(GF_ERR_INVALID_ARG, "dparams needs the transform guide");
  if (misaligned(I_lo) || misaligned(p_lo) || misaligned(I_hi) || misaligned(dq_hi) ||
      misaligned(dI_lo) || misaligned(dp_lo) || misaligned(dI_hi) || misaligned(q_hi) ||
      misaligned(ws))
    return fail(GF_ERR_INVALID_ARG, "tensor pointers must be 16-byte aligned");
  const size_t need = with_forward ? std::max(p.ws_fwd, p.ws_bwd) : p.ws_bwd;
  if (!ws || ws_bytes < need)
    return fail(GF_ERR_WORKSPACE, std::string("workspace smaller than gf_workspace_size(desc, guide, ") +
                                      (with_forward ? "2" : "1") + ") = " + std::to_string(need));
  gf::BwdArgs a{I_lo, p_lo, I_hi, dq_hi, eps, eps_count, dI_lo, dp_lo, deps, dparams, dI_hi,
                static_cast<char*>(ws), with_forward ? q_hi : nullptr};
  hipError_t e = gf::launch_backward(p, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(GF_ERR_HIP, hipGetErrorString(e));
  return GF_OK;
}
}  // namespace

extern "C" {

int32_t gf_backward(const gf_desc_t* desc, const gf_guide_t* guide, const void* I_lo,
                    const void* p_lo, const void* I_hi, const float* eps, int32_t eps_count,
                    const void* dq_hi, float* dI_lo, float* dp_lo, void* dI_hi, float* deps,
                    float* dparams, void* ws, size_t ws_bytes, void* stream) {
  return run_backward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, nullptr, dI_lo,
                      dp_lo, dI_hi, deps, dparams, ws, ws_bytes, stream, false);
}

int32_t gf_forward_backward(const gf_desc_t* desc, const gf_guide_t* guide, const void* I_lo,
                            const void* p_lo, const void* I_hi, const float* eps,
                            int32_t eps_count, const void* dq_hi, void* q_hi, float* dI_lo,
                            float* dp_lo, void* dI_hi, float* deps, float* dparams, void* ws,
                            size_t ws_bytes, void* stream) {
  return run_backward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, q_hi, dI_lo, dp_lo,
                      dI_hi, deps, dparams, ws, ws_bytes, stream, true);
}

size_t gf_conv_param_count(int32_t c, int32_t hidden) {
  if (c < 1 || c > gf::kConvMaxC || hidden < 1 || hidden > gf::kConvMaxK) return 0;
  return (size_t)gf::conv_param_count(c, hidden);
}

}  // extern "C"

namespace gf {
namespace {
// Plan of the convolutional layer: the high-res kernels' plan (the radius of
// the box filter plays no part, the dilation lives in cp->r) and the
// low-res workspace appended to that plan's layout.
int make_conv_plan(const gf_desc_t* d, const gf_conv_t* cv, ConvPlan* cp, const char** why) {
  static thread_local std::string msg;
  auto bad = [&](int code, const std::string& m) {
    msg = m;
    *why = msg.c_str();
    return code;
  };
  if (!d) return bad(GF_ERR_INVALID_ARG, "desc is NULL");
  if (!cv) return bad(GF_ERR_INVALID_ARG, "conv is NULL");
  if (d->r < 1) return bad(GF_ERR_INVALID_ARG, "dilation r must be >= 1");
  if (d->r > 1 << 20) return bad(GF_ERR_UNSUPPORTED, "dilation too large");
  if (d->c < 1 || d->c > kConvMaxC) return bad(GF_ERR_UNSUPPORTED, "channels must be 1..4");
  if (cv->hidden < 1 || cv->hidden > kConvMaxK)
    return bad(GF_ERR_UNSUPPORTED, "hidden width must be 1..16");
  if (!cv->params) return bad(GF_ERR_INVALID_ARG, "conv params is NULL");
  if (!(cv->slope >= 0.f) || !(cv->slope <= 1.f))
    return bad(GF_ERR_INVALID_ARG, "leaky ReLU slope must be in [0, 1]");
  gf_desc_t d1 = *d;
  d1.r = 1;
  int st = make_plan(&d1, nullptr, &cp->p, why);
  if (st != GF_OK) return st;
  if ((double)d->n * d->h_lo * d->w_lo > 2.0e9) return bad(GF_ERR_UNSUPPORTED, "problem too large");
  cp->r = d->r;
  cp->K = cv->hidden;
  cp->slope = cv->slope;
  cp->params = cv->params;
  cp->nparam = conv_param_count(d->c, cv->hidden);
  const long long npix = (long long)d->n * d->h_lo * d->w_lo;
  const long long tiles = (npix + kConvTile - 1) / kConvTile;
  cp->blk_grid = (int)std::min<long long>(tiles, kConvBlocks);
  cp->ab_grid = (int)std::min<long long>(((long long)d->h_lo * d->w_lo + 255) / 256, kConvAbGrid);
  const size_t lo = align_up((size_t)cp->p.planes * d->h_lo * d->w_lo * sizeof(float), 256);
  size_t o = align_up(std::max(cp->p.ws_fwd, cp->p.ws_bwd), 256);
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes, 256);
    return at;
  };
  cp->off_A = take(lo);
  cp->off_B = take(lo);
  cp->ws_fwd = o;
  cp->off_mI = take(lo);
  cp->off_mP = take(lo);
  cp->off_cov = take(lo);
  cp->off_var = take(lo);
  cp->off_dAb = take(lo);
  cp->off_dBb = take(lo);
  cp->off_dA = take(lo);
  cp->off_dB = take(lo);
  cp->off_gmI = take(lo);
  cp->off_gmP = take(lo);
  cp->off_gcov = take(lo);
  cp->off_gvar = take(lo);
  cp->off_part = take((size_t)cp->blk_grid * cp->nparam * sizeof(float));
  cp->off_partab = take((size_t)cp->p.planes * cp->ab_grid * 9 * sizeof(float));
  cp->ws_bwd = o;
  return GF_OK;
}

ConvArgs conv_args(const ConvPlan& cp, const gf_desc_t* d, const void* I_lo, const void* p_lo,
                   char* ws, bool backward) {
  auto f = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
  ConvArgs a{};
  a.I_lo = I_lo;
  a.p_lo = p_lo;
  a.params = cp.params;
  a.n = d->n;
  a.c = d->c;
  a.h = d->h_lo;
  a.w = d->w_lo;
  a.r = cp.r;
  a.K = cp.K;
  a.nparam = cp.nparam;
  a.mean_ab = d->mean_ab;
  a.slope = cp.slope;
  a.abar = f(cp.p.off_abar);
  a.bbar = f(cp.p.off_bbar);
  // without the window means, A and b are the upsampled planes themselves
  a.A = d->mean_ab ? f(cp.off_A) : a.abar;
  a.B = d->mean_ab ? f(cp.off_B) : a.bbar;
  if (backward) {
    a.mI = f(cp.off_mI);
    a.mP = f(cp.off_mP);
    a.cov = f(cp.off_cov);
    a.var = f(cp.off_var);
    a.dAb = f(cp.off_dAb);
    a.dBb = f(cp.off_dBb);
    a.dA = d->mean_ab ? f(cp.off_dA) : a.dAb;
    a.dB = d->mean_ab ? f(cp.off_dB) : a.dBb;
    a.gmI = f(cp.off_gmI);
    a.gmP = f(cp.off_gmP);
    a.gcov = f(cp.off_gcov);
    a.gvar = f(cp.off_gvar);
    a.part = f(cp.off_part);
    a.partab = f(cp.off_partab);
  }
  a.blk_grid = cp.blk_grid;
  a.ab_grid = cp.ab_grid;
  return a;
}
}  // namespace
}  // namespace gf

extern "C" {

size_t gf_conv_workspace_size(const gf_desc_t* desc, const gf_conv_t* conv, int32_t backward) {
  gf::ConvPlan cp;
  const char* why = nullptr;
  if (gf::make_conv_plan(desc, conv, &cp, &why) != GF_OK) return 0;
  return backward ? cp.ws_bwd : cp.ws_fwd;
}

int32_t gf_conv_forward(const gf_desc_t* desc, const gf_conv_t* conv, const void* I_lo,
                        const void* p_lo, const void* I_hi, void* q_hi, void* ws,
                        size_t ws_bytes, void* stream) {
  gf::g_detail.clear();
  gf::ConvPlan cp;
  const char* why = nullptr;
  int st = gf::make_conv_plan(desc, conv, &cp, &why);
  if (st != GF_OK) return fail(st, why);
  if (!I_lo || !p_lo || !I_hi || !q_hi) return fail(GF_ERR_INVALID_ARG, "a required pointer is NULL");
  if (misaligned(I_lo) || misaligned(p_lo) || misaligned(I_hi) || misaligned(q_hi) ||
      misaligned(ws) || misaligned(conv->params))
    return fail(GF_ERR_INVALID_ARG, "tensor pointers must be 16-byte aligned");
  if (!ws || ws_bytes < cp.ws_fwd)
    return fail(GF_ERR_WORKSPACE, "workspace smaller than gf_conv_workspace_size(desc, conv, 0) = " +
                                      std::to_string(cp.ws_fwd));
  char* w = static_cast<char*>(ws);
  const gf::ConvArgs a = gf::conv_args(cp, desc, I_lo, p_lo, w, false);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipErrorInvalidValue;
  switch (desc->io_dtype) {
    case GF_F32: e = gf::launch_conv_forward_f32(cp, a, I_hi, q_hi, w, s); break;
    case GF_F16: e = gf::launch_conv_forward_f16(cp, a, I_hi, q_hi, w, s); break;
    case GF_BF16: e = gf::launch_conv_forward_bf16(cp, a, I_hi, q_hi, w, s); break;
  }
  if (e != hipSuccess) return fail(GF_ERR_HIP, hipGetErrorString(e));
  return GF_OK;
}

int32_t gf_conv_backward(const gf_desc_t* desc, const gf_conv_t* conv, const void* I_lo,
                         const void* p_lo, const void* I_hi, const void* dq_hi, float* dI_lo,
                         float* dp_lo, void* dI_hi, float* dparams, void* ws, size_t ws_bytes,
                         void* stream) {
  gf::g_detail.clear();
  gf::ConvPlan cp;
  const char* why = nullptr;
  int st = gf::make_conv_plan(desc, conv, &cp, &why);
  if (st != GF_OK) return fail(st, why);
  if (!I_lo || !p_lo || !I_hi || !dq_hi)
    return fail(GF_ERR_INVALID_ARG, "a required pointer is NULL");
  if (misaligned(I_lo) || misaligned(p_lo) || misaligned(I_hi) || misaligned(dq_hi) ||
      misaligned(dI_lo) || misaligned(dp_lo) || misaligned(dI_hi) || misaligned(dparams) ||
      misaligned(ws) || misaligned(conv->params))
    return fail(GF_ERR_INVALID_ARG, "tensor pointers must be 16-byte aligned");
  if (!ws || ws_bytes < cp.ws_bwd)
    return fail(GF_ERR_WORKSPACE, "workspace smaller than gf_conv_workspace_size(desc, conv, 1) = " +
                                      std::to_string(cp.ws_bwd));
  char* w = static_cast<char*>(ws);
  gf::ConvArgs a = gf::conv_args(cp, desc, I_lo, p_lo, w, true);
  a.dI_lo = dI_lo;
  a.dp_lo = dp_lo;
  a.dparams = dparams;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipErrorInvalidValue;
  switch (desc->io_dtype) {
    case GF_F32: e = gf::launch_conv_backward_f32(cp, a, I_hi, dq_hi, dI_hi, w, s); break;
    case GF_F16: e = gf::launch_conv_backward_f16(cp, a, I_hi, dq_hi, dI_hi, w, s); break;
    case GF_BF16: e = gf::launch_conv_backward_bf16(cp, a, I_hi, dq_hi, dI_hi, w, s); break;
  }
  if (e != hipSuccess) return fail(GF_ERR_HIP, hipGetErrorString(e));
  return GF_OK;
}

int32_t gf_downsample(int32_t n, int32_t c, int32_t h_hi, int32_t w_hi, int32_t h_lo,
                      int32_t w_lo, int32_t io_dtype, const void* I_hi, void* I_lo,
                      void* stream) {
  gf::g_detail.clear();
  if (n < 1 || c < 1 || h_hi < 1 || w_hi < 1 || h_lo < 1 || w_lo < 1)
    return fail(GF_ERR_INVALID_ARG, "sizes must be >= 1");
  if (h_lo > h_hi || w_lo > w_hi)
    return fail(GF_ERR_INVALID_ARG, "low-res size must not exceed high-res size");
  if (gf::dtype_size(io_dtype) == 0) return fail(GF_ERR_INVALID_ARG, "unknown io_dtype");
  if (!I_hi || !I_lo) return fail(GF_ERR_INVALID_ARG, "a required pointer is NULL");
  if (misaligned(I_hi) || misaligned(I_lo))
    return fail(GF_ERR_INVALID_ARG, "tensor pointers must be 16-byte aligned");
  const long long planes = (long long)n * c;
  if (planes > 65535 || h_lo > 65535 || (double)planes * h_hi * w_hi > 9.0e15)
    return fail(GF_ERR_UNSUPPORTED, "problem too large");
  // low-res columns per workgroup: at most 256, fewer while the high-res
  // columns they cover exceed the LDS row buffer, and fewer (down to 4)
  // while the grid would not give the chip a few workgroups per CU (a 64 x 64
  // I_l under a 3072^2 I_h is 192 rows x planes otherwise)
  int jc = std::min(256, (int)w_lo);
  auto span = [&](int j) { return (int)(((long long)j * w_hi + w_lo - 1) / w_lo) + 1; };
  while (jc > 1 && span(jc) > gf::kDownMaxSpan) jc /= 2;
  auto wgs = [&](int j) { return planes * h_lo * (long long)((w_lo + j - 1) / j); };
  while (jc > 4 && wgs(jc) < 2048) jc /= 2;
  if (span(jc) > gf::kDownMaxSpan)
    return fail(GF_ERR_UNSUPPORTED, "a low-res pixel covers more than 8191 high-res columns");
  gf::DownArgs a{I_hi, I_lo, (int)planes, h_hi, w_hi, h_lo, w_lo, jc, span(jc)};
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipErrorInvalidValue;
  switch (io_dtype) {
    case GF_F32: e = gf::launch_downsample_f32(a, s); break;
    case GF_F16: e = gf::launch_downsample_f16(a, s); break;
    case GF_BF16: e = gf::launch_downsample_bf16(a, s); break;
  }
  if (e != hipSuccess) return fail(GF_ERR_HIP, hipGetErrorString(e));
  return GF_OK;
}

const char* gf_status_string(int32_t status) {
  switch (status) {
    case GF_OK: return "GF_OK";
    case GF_ERR_INVALID_ARG: return "GF_ERR_INVALID_ARG";
    case GF_ERR_UNSUPPORTED: return "GF_ERR_UNSUPPORTED";
    case GF_ERR_WORKSPACE: return "GF_ERR_WORKSPACE";
    case GF_ERR_HIP: return "GF_ERR_HIP";
  }
  return "GF_ERR_UNKNOWN";
}

const char* gf_last_error_detail(void) { return gf::g_detail.c_str(); }

int32_t gf_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(gf::g_prof_mu);
  gf::prof_clear();
  gf::g_prof_on = on != 0;
  // records of a few hundred launches without creating events on the way
  while (gf::g_prof_on && gf::g_ev_pool.size() < 2048) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) break;
    gf::g_ev_pool.push_back(e);
  }
  return GF_OK;
}

int32_t gf_profile_read(char (*names)[48], double* ms, int32_t* launches, int32_t cap) {
  std::lock_guard<std::mutex> lk(gf::g_prof_mu);
  std::vector<std::string> keys;
  std::vector<double> tot;
  std::vector<int> cnt;
  for (auto& r : gf::g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) continue;
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) continue;
    size_t k = 0;
    while (k < keys.size() && keys[k] != r.name) ++k;
    if (k == keys.size()) {
      keys.push_back(r.name);
      tot.push_back(0.0);
      cnt.push_back(0);
    }
    tot[k] += t;
    cnt[k] += 1;
  }
  gf::prof_clear();
  const int m = (int)keys.size();
  for (int k = 0; k < m && k < cap; ++k) {
    if (names) {
      strncpy(names[k], keys[k].c_str(), 47);
      names[k][47] = '\0';
    }
    if (ms) ms[k] = tot[k];
    if (launches) launches[k] = cnt[k];
  }
  return m;
}

}  // extern "C"

// ------------------------------------------------------------ tile-shape table and autotuner

namespace gf {
namespace {
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, TuneVal>> g_tune;

bool same_key(const TuneKey& a, const TuneKey& b) {
  return a.dtype == b.dtype && a.S == b.S && a.r == b.r && a.gmode == b.gmode &&
         a.mean_ab == b.mean_ab;
}

bool tune_erase(const TuneKey& k) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (size_t i = 0; i < g_tune.size(); ++i)
    if (same_key(g_tune[i].first, k)) {
      g_tune.erase(g_tune.begin() + i);
      return true;
    }
  return false;
}
}  // namespace

bool tune_lookup(const TuneKey& k, TuneVal* v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune)
    if (same_key(e.first, k)) {
      *v = e.second;
      return true;
    }
  return false;
}

void tune_store(const TuneKey& k, const TuneVal& v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune)
    if (same_key(e.first, k)) {
      e.second = v;
      return;
    }
  g_tune.push_back({k, v});
}
}  // namespace gf

extern "C" {

size_t gf_tune_export(char* buf, size_t cap) {
  std::string out;
  {
    std::lock_guard<std::mutex> lk(gf::g_tune_mu);
    for (auto& e : gf::g_tune) {
      char line[160];
      snprintf(line, sizeof line, "%d %d %d %d %d : %d %d %d %d\n", e.first.dtype, e.first.S,
               e.first.r, e.first.gmode, e.first.mean_ab, e.second.coTR, e.second.loTR,
               e.second.RB, e.second.bh);
      out += line;
    }
  }
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, out.size());
    memcpy(buf, out.data(), n);
    buf[n] = '\0';
  }
  return out.size();
}

int32_t gf_tune_import(const char* text) {
  gf::g_detail.clear();
  if (!text) return fail(GF_ERR_INVALID_ARG, "text is NULL");
  std::vector<std::pair<gf::TuneKey, gf::TuneVal>> parsed;
  const char* p = text;
  int lineno = 0;
  while (*p) {
    const char* e = strchr(p, '\n');
    std::string line(p, e ? (size_t)(e - p) : strlen(p));
    p = e ? e + 1 : p + line.size();
    ++lineno;
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    gf::TuneKey k;
    gf::TuneVal v;
    char colon = 0;
    int used = 0;
    if (sscanf(line.c_str(), " %d %d %d %d %d %c %d %d %d %d %n", &k.dtype, &k.S, &k.r, &k.gmode,
               &k.mean_ab, &colon, &v.coTR, &v.loTR, &v.RB, &v.bh, &used) != 10 ||
        colon != ':' || line.find_first_not_of(" \t\r", used) != std::string::npos ||
        v.coTR < 1 || v.loTR < 1 || v.RB < 1 || v.bh < 2)
      return fail(GF_ERR_INVALID_ARG, "malformed tuning line " + std::to_string(lineno));
    parsed.push_back({k, v});
  }
  for (auto& kv : parsed) gf::tune_store(kv.first, kv.second);
  return GF_OK;
}

int32_t gf_autotune(const gf_desc_t* desc, const gf_guide_t* guide, const void* I_lo,
                    const void* p_lo, const void* I_hi, const float* eps, int32_t eps_count,
                    void* q_hi, const void* dq_hi, float* dI_lo, float* dp_lo, void* dI_hi,
                    float* deps, float* dparams, void* ws, size_t ws_bytes, int32_t iters,
                    void* stream) {
  gf::g_detail.clear();
  gf::Plan p0;
  const char* why = nullptr;
  int st = gf::make_plan(desc, guide, &p0, &why);
  if (st != GF_OK) return fail(st, why);
  if (iters < 1 || iters > 1000) return fail(GF_ERR_INVALID_ARG, "iters must be 1..1000");
  const gf::TuneKey key{desc->io_dtype, p0.S, p0.r, p0.gmode, desc->mean_ab};
  gf::TuneVal saved;
  const bool had = gf::tune_lookup(key, &saved);
  // candidates, tried index by index (kernel k takes its k-th list)
  const int lo_rows[] = {16, 32, 64, 128};
  const int apply_rows[] = {4, 8, 16, 32};
  const int bwd_rows[] = {2, 4, 8, 2};
  const char* names[4] = {"gf_coef", "gf_bwd_lo", "gf_apply", "gf_bwd_hi"};
  double best[4] = {1e30, 1e30, 1e30, 1e30};
  gf::TuneVal pick{p0.coTR, p0.loTR, p0.RB, p0.bh};
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto restore = [&]() {
    if (had)
      gf::tune_store(key, saved);
    else
      gf::tune_erase(key);
  };
  for (int i = 0; i < 4; ++i) {
    const gf::TuneVal v{lo_rows[i], lo_rows[i], apply_rows[i], bwd_rows[i]};
    gf::tune_store(key, v);
    gf::Plan p;
    if (gf::make_plan(desc, guide, &p, &why) != GF_OK || p.ws_bwd > ws_bytes ||
        p.ws_fwd > ws_bytes)
      continue;
    auto step = [&]() {
      int a = gf_forward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, q_hi, ws, ws_bytes,
                         stream);
      if (a != GF_OK) return a;
      return gf_backward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, dI_lo, dp_lo,
                         dI_hi, deps, dparams, ws, ws_bytes, stream);
    };
    int a = step();  // warm-up
    if (a != GF_OK) {
      restore();
      return a;
    }
    gf_profile_enable(1);
    for (int it = 0; it < iters && a == GF_OK; ++it) a = step();
    char nm[16][48];
    double ms[16];
    int32_t cnt[16];
    const int m = gf_profile_read(nm, ms, cnt, 16);
    gf_profile_enable(0);
    if (a != GF_OK) {
      restore();
      return a;
    }
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < m && j < 16; ++j)
        if (strcmp(nm[j], names[k]) == 0 && cnt[j] > 0) {
          const double avg = ms[j] / cnt[j];
          if (avg < best[k]) {
            best[k] = avg;
            if (k == 0) pick.coTR = v.coTR;
            if (k == 1) pick.loTR = v.loTR;
            if (k == 2) pick.RB = v.RB;
            if (k == 3) pick.bh = v.bh;
          }
        }
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    restore();
    return fail(GF_ERR_HIP, "stream synchronisation failed");
  }
  gf::tune_store(key, pick);
  gf::Plan p;
  if (gf::make_plan(desc, guide, &p, &why) != GF_OK || p.ws_bwd > ws_bytes) {
    restore();
    return fail(GF_ERR_WORKSPACE, "no tuned shape fits the workspace");
  }
  return GF_OK;
}

}  // extern "C"

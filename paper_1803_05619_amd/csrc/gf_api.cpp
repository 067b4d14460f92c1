// C ABI of the guided filtering layer: argument checks, launch planning,
// workspace layout and kernel timing.  Every check runs on the host before
// any HIP call, so invalid input is reported without touching a device.

#include <hip/hip_runtime.h>
#include <stdint.h>
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
  if (dtype_size(d->io_dtype) == 0) return bad(GF_ERR_INVALID_ARG, "unknown io_dtype");
  if (d->h_hi % d->h_lo || d->w_hi % d->w_lo || d->h_hi / d->h_lo != d->w_hi / d->w_lo)
    return bad(GF_ERR_UNSUPPORTED, "high/low size ratio must be one integer factor for both axes");
  const int S = d->h_hi / d->h_lo;
  if (S != 1 && S != 2 && S != 4 && S != 8)
    return bad(GF_ERR_UNSUPPORTED, "upsampling factor must be 1, 2, 4 or 8");
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
  q.dtype = d->io_dtype;
  q.S = S;
  q.xcd = env_int("GF_XCD", 0) != 0 ? 1 : 0;  // measured slower on MI355X: off by default
  q.planes = d->n * d->c;
  // elements per lane-load on the high-res side: 16 bytes, at least S (a
  // lane then covers whole low-res columns), 1 when W is not a multiple
  // (guided path: the high-res kernels read the float guide plane G_h)
  int V = gmode == GF_GUIDE_IDENTITY ? 16 / dtype_size(d->io_dtype) : 4;
  if (V < S) V = S;
  q.VEC = (q.W % V == 0) ? V : 1;

  const int r = q.r;
  if (r > kMaxRadius) return bad(GF_ERR_UNSUPPORTED, "radius above 10 is not supported");
  const int hal = q.mean_ab ? 2 * r : r;  // halo of the coefficient walker
  const size_t KRc = walker_ring_rows(r, kWalkBlock, kCoefRingPow2Max);
  const size_t KRb = walker_ring_rows(r, kWalkBlock, kBwdLoRingPow2Max);
  // rows per wave: long enough to amortise the 2*halo warm-up rows
  q.coTR = r <= 2 ? 32 : 64;
  if (env_int("GF_LO_ROWS", 0) > 0) q.coTR = env_int("GF_LO_ROWS", 0);
  q.co_nx = (q.w + (64 - 2 * hal) - 1) / (64 - 2 * hal);
  q.co_ny = (q.h + q.coTR - 1) / q.coTR;
  q.coLDS = 64 * (16 * KRc + 24 * kWalkBlock);  // (g,p), (A,b) rings + row buffers
  q.loTR = q.coTR;
  q.lo_nx = (q.w + (64 - 4 * r) - 1) / (64 - 4 * r);
  q.lo_ny = (q.h + q.loTR - 1) / q.loTR;
  q.loLDS = 64 * (32 * KRb + 40 * kWalkBlock);  // input and X rings + row buffers

  // Launch-shape overrides (tuning experiments): GF_APPLY_ROWS = high-res rows
  // per apply thread, GF_BWD_BH = low-res rows per backward high-res block.
  const int rows_env = env_int("GF_APPLY_ROWS", 0), bh_env = env_int("GF_BWD_BH", 0);
  // Short walks keep DRAM streams sequential (8 rows per thread measured
  // best on MI355X for the 4 x 3 x 2048 x 3072 workload): two low-res row
  // blocks at S = 4, one at S = 8.
  q.RB = S >= 8 ? S : 8;
  if (rows_env > 0) q.RB = ((rows_env + S - 1) / S) * S;
  q.nrb = (q.H + q.RB - 1) / q.RB;
  q.nxv = q.W / q.VEC;

  // Backward high-res blocks of 2 low-res rows (2 S high-res rows): short
  // walks stream best; the partial planes' extra border rows cost less.
  q.bh = 2;
  if (bh_env >= 2) q.bh = bh_env;
  q.tw = 64 * q.VEC / S;
  q.nby = (q.h + q.bh - 1) / q.bh;
  q.nbx = (q.W + 64 * q.VEC - 1) / (64 * q.VEC);
  q.ublk_floats = (size_t)2 * (q.bh + 2) * (q.tw + 2);

  const size_t lo_plane = (size_t)q.planes * q.h * q.w * sizeof(float);
  q.off_abar = 0;
  q.off_bbar = align_up(lo_plane, 256);
  q.ws_fwd = q.off_bbar + align_up(lo_plane, 256);
  q.off_u = align_up(lo_plane, 256);
  const size_t ubytes = (size_t)q.planes * q.nby * q.nbx * q.ublk_floats * sizeof(float);
  q.off_eps = q.off_u + align_up(ubytes, 256);
  q.ws_bwd = q.off_eps + align_up((size_t)q.planes * q.lo_nx * q.lo_ny * sizeof(float), 256);
  if (gmode != GF_GUIDE_IDENTITY) {
    // guided path: the guide planes and the transform's reductions follow the
    // identity layout (a superset is allocated for both directions)
    const size_t lo = (size_t)q.planes * q.h * q.w * sizeof(float);
    const size_t hi = (size_t)q.planes * q.H * q.W * sizeof(float);
    auto chunks = [](long long P) { return (int)std::min<long long>(64, (P + 16383) / 16384); };
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

void prof_clear() {
  for (auto& r : g_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
  if (g_pending_ev) (void)hipEventDestroy(g_pending_ev);
  g_pending_ev = nullptr;
}
}  // namespace

void prof_begin(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  hipEvent_t ev;
  if (hipEventCreate(&ev) != hipSuccess) return;
  (void)hipEventRecord(ev, s);
  g_pending_name = name;
  g_pending_ev = ev;
}

void prof_end(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on || !g_pending_ev) return;
  hipEvent_t ev;
  if (hipEventCreate(&ev) != hipSuccess) return;
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

int32_t gf_backward(const gf_desc_t* desc, const gf_guide_t* guide, const void* I_lo,
                    const void* p_lo, const void* I_hi, const float* eps, int32_t eps_count,
                    const void* dq_hi, float* dI_lo, float* dp_lo, void* dI_hi, float* deps,
                    float* dparams, void* ws, size_t ws_bytes, void* stream) {
  gf::g_detail.clear();
  gf::Plan p;
  const char* why = nullptr;
  int st = gf::make_plan(desc, guide, &p, &why);
  if (st != GF_OK) return fail(st, why);
  if (!I_lo || !p_lo || !I_hi || !eps || !dq_hi)
    return fail(GF_ERR_INVALID_ARG, "a required pointer is NULL");
  if (eps_count != 1 && eps_count != desc->n)
    return fail(GF_ERR_INVALID_ARG, "eps_count must be 1 or n");
  if (dparams && p.gmode != GF_GUIDE_TRANSFORM)
    return fail(GF_ERR_INVALID_ARG, "dparams needs the transform guide");
  if (misaligned(I_lo) || misaligned(p_lo) || misaligned(I_hi) || misaligned(dq_hi) ||
      misaligned(dI_lo) || misaligned(dp_lo) || misaligned(dI_hi) || misaligned(ws))
    return fail(GF_ERR_INVALID_ARG, "tensor pointers must be 16-byte aligned");
  if (!ws || ws_bytes < p.ws_bwd)
    return fail(GF_ERR_WORKSPACE, "workspace smaller than gf_workspace_size(desc, guide, 1) = " +
                                      std::to_string(p.ws_bwd));
  gf::BwdArgs a{I_lo, p_lo, I_hi, dq_hi, eps, eps_count, dI_lo, dp_lo, deps, dparams, dI_hi,
                static_cast<char*>(ws)};
  hipError_t e = gf::launch_backward(p, a, static_cast<hipStream_t>(stream));
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

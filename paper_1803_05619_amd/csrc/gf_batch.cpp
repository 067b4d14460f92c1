// Batched plans: many independent guided-filter problems (different sizes,
// factors, radii and eps) as one launch per phase and launch class.  The
// host validates every item, derives its launch shapes with the same
// planner as the single-problem calls, groups the items by the template
// parameters of the kernels (radius and mean_ab for the low-res phases, the
// factor and vector width for the high-res ones), and uploads one table per
// class: the items' arguments and the first tile of each item.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "gf_internal.h"

struct gf_plan {
  int dtype = 0;
  int count = 0;
  int device = 0;
  bool all_q = true, all_dq = true;
  gf::BatchLaunch launch;
  char* dmem = nullptr;
  size_t ws_bytes = 0;
  hipStream_t cap = nullptr;
  struct Graph {
    int mode;
    void* ws;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
};

namespace gf {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace-relative pointer as the multi kernels expect it (offset + 1).
template <typename T>
T* ws_rel(size_t off) {
  return reinterpret_cast<T*>(static_cast<uintptr_t>(off) + 1);
}

bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) != 0; }

struct Geo {
  Plan p;
  size_t off_abar, off_bbar, off_u, off_eps, off_x;
  long long t_coef, t_apply, t_bwd_hi, t_bwd_lo;
};

struct Member {
  int item;
  long long tiles;
};

using ClassMap = std::map<std::pair<int, int>, std::vector<Member>>;

// Device table of one class: base[n] then MultiItem<Args>[n] (256-aligned).
template <typename Args>
size_t class_bytes(size_t n) {
  return align_up(n * sizeof(long long), 256) + align_up(n * sizeof(MultiItem<Args>), 256);
}

template <typename Args, typename MakeArgs, typename Dims>
void build_classes(const ClassMap& cm, int kind, std::vector<char>& host, size_t& off,
                   char* dmem, MakeArgs make_args, Dims dims, size_t (*lds)(const Geo&),
                   const std::vector<Geo>& geo, std::vector<BatchClass>& out) {
  for (auto& kv : cm) {
    std::vector<Member> mem = kv.second;
    // largest items first: their tiles start first, the small ones fill the tail
    std::stable_sort(mem.begin(), mem.end(),
                     [](const Member& a, const Member& b) { return a.tiles > b.tiles; });
    const size_t n = mem.size();
    const size_t base_off = off;
    const size_t items_off = off + align_up(n * sizeof(long long), 256);
    long long* base = reinterpret_cast<long long*>(host.data() + base_off);
    MultiItem<Args>* items = reinterpret_cast<MultiItem<Args>*>(host.data() + items_off);
    long long total = 0;
    for (size_t i = 0; i < n; ++i) {
      const int k = mem[i].item;
      base[i] = total;
      MultiItem<Args> it{};
      it.a = make_args(k);
      dims(geo[k], it.nx, it.ny);
      it.base = total;
      items[i] = it;
      total += mem[i].tiles;
    }
    off += class_bytes<Args>(n);
    BatchClass c{};
    c.kind = kind;
    if (kind == kClassCoef || kind == kClassBwdLo) {
      c.R = kv.first.first;
      c.MAB = kv.first.second % 2;
      c.wide = kv.first.second / 2;
    } else {  // high-res key: (S, 2 VEC + corner alignment)
      c.S = kv.first.first;
      c.VEC = kv.first.second / 2;
      c.AC = kv.first.second % 2;
    }
    c.hw = geo[mem[0].item].p.hw;  // high-res classes: one dtype and factor, one value
    c.lds = 0;  // the largest of the class's items
    if (lds)
      for (const Member& m : mem) c.lds = std::max(c.lds, lds(geo[m.item]));
    c.m.base = reinterpret_cast<const long long*>(dmem + base_off);
    c.m.items = dmem + items_off;
    c.m.count = (int)n;
    c.m.total = total;
    c.m.ws = nullptr;
    // grid: one workgroup per tile, or a persistent grid-stride grid when
    // GF_BATCH_WGS caps it
    const char* cap = getenv("GF_BATCH_WGS");
    const long long wcap = cap ? atoll(cap) : 0;
    c.m.grid = (int)((wcap > 0 && wcap < total) ? wcap : total);
    out.push_back(c);
  }
}

int create(const gf_item_t* items, int count, gf_plan** out) {
  if (!out) return set_error(GF_ERR_INVALID_ARG, "plan is NULL");
  *out = nullptr;
  if (!items || count < 1) return set_error(GF_ERR_INVALID_ARG, "need at least one item");
  std::vector<Geo> geo(count);
  size_t ws = 0;
  bool all_q = true, all_dq = true;
  for (int k = 0; k < count; ++k) {
    const gf_item_t& it = items[k];
    const std::string tag = "item " + std::to_string(k) + ": ";
    const char* why = nullptr;
    const int st = make_plan(&it.d, nullptr, &geo[k].p, &why);
    if (st != GF_OK) return set_error(st, tag + why);
    if (geo[k].p.gen)
      return set_error(GF_ERR_UNSUPPORTED,
                       tag + "batched plans take one integer factor 1, 2, 4 or 8 for both "
                             "axes (other ratios: gf_forward / gf_backward)");
    if (it.d.io_dtype != items[0].d.io_dtype)
      return set_error(GF_ERR_INVALID_ARG, tag + "io_dtype differs from item 0");
    if (!(it.eps >= 0.f) || !isfinite(it.eps))
      return set_error(GF_ERR_INVALID_ARG, tag + "eps must be finite and >= 0");
    if (!it.I_lo || !it.p_lo || !it.I_hi)
      return set_error(GF_ERR_INVALID_ARG, tag + "a required pointer is NULL");
    if (misaligned(it.I_lo) || misaligned(it.p_lo) || misaligned(it.I_hi) ||
        misaligned(it.q_hi) || misaligned(it.dq_hi) || misaligned(it.dI_lo) ||
        misaligned(it.dp_lo) || misaligned(it.dI_hi))
      return set_error(GF_ERR_INVALID_ARG, tag + "tensor pointers must be 16-byte aligned");
    all_q = all_q && it.q_hi;
    all_dq = all_dq && it.dq_hi;
    Geo& g = geo[k];
    const Plan& p = g.p;
    const size_t lo_plane = (size_t)p.planes * p.h * p.w * sizeof(float);
    g.off_abar = ws;
    ws += align_up(lo_plane, 256);
    g.off_bbar = ws;
    ws += align_up(lo_plane, 256);
    g.off_u = ws;
    ws += align_up((size_t)p.planes * p.nby * p.nbx * p.ublk_floats * sizeof(float), 256);
    g.off_eps = ws;
    ws += align_up((size_t)p.planes * p.lo_nx * p.lo_ny * sizeof(float), 256);
    g.off_x = ws;  // the wide backward's X planes
    if (p.wide_lo || (p.wide_co && p.mean_ab))
      ws += align_up((size_t)p.planes * p.h * p.w * wide_x_floats(p) * sizeof(float), 256);
    g.t_coef = (long long)p.co_nx * p.co_ny * p.planes;
    g.t_bwd_lo = (long long)p.lo_nx * p.lo_ny * p.planes;
    g.t_apply = ((long long)p.planes * p.nrb * p.nxv + 255) / 256;
    g.t_bwd_hi = (long long)p.nbx * p.nby * p.planes;
  }
  ClassMap cm_coef, cm_lo, cm_hi;
  int n_eps = 0;
  for (int k = 0; k < count; ++k) {
    const Plan& p = geo[k].p;
    // low-res classes: (radius, mean_ab + 2 x walker kind)
    cm_coef[{p.r, p.mean_ab + 2 * p.wide_co}].push_back({k, geo[k].t_coef});
    cm_lo[{p.r, p.mean_ab + 2 * p.wide_lo}].push_back({k, geo[k].t_bwd_lo});
    cm_hi[{p.S, 2 * p.VEC + p.ac}].push_back({k, geo[k].t_bwd_hi});
    if (items[k].deps) ++n_eps;
  }
  ClassMap cm_apply;
  for (int k = 0; k < count; ++k)
    cm_apply[{geo[k].p.S, 2 * geo[k].p.VEC + geo[k].p.ac}].push_back({k, geo[k].t_apply});

  // device table layout: eps values, four class families, eps items
  size_t total = align_up((size_t)count * sizeof(float), 256);
  for (auto& kv : cm_coef) total += class_bytes<CoefArgs>(kv.second.size());
  for (auto& kv : cm_apply) total += class_bytes<ApplyArgs>(kv.second.size());
  for (auto& kv : cm_hi) total += class_bytes<BwdHiArgs>(kv.second.size());
  for (auto& kv : cm_lo) total += class_bytes<BwdLoArgs>(kv.second.size());
  const size_t eps_items_off = total;
  total += align_up((size_t)std::max(n_eps, 1) * sizeof(EpsItem), 256);

  gf_plan* pl = new gf_plan();
  pl->dtype = items[0].d.io_dtype;
  pl->count = count;
  pl->all_q = all_q;
  pl->all_dq = all_dq;
  pl->ws_bytes = std::max<size_t>(ws, 256);
  if (hipGetDevice(&pl->device) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&pl->dmem), total) != hipSuccess) {
    delete pl;
    return set_error(GF_ERR_HIP, "device table allocation failed");
  }
  std::vector<char> host(total, 0);
  float* eps_host = reinterpret_cast<float*>(host.data());
  for (int k = 0; k < count; ++k) eps_host[k] = items[k].eps;
  const float* eps_dev = reinterpret_cast<const float*>(pl->dmem);
  size_t off = align_up((size_t)count * sizeof(float), 256);

  build_classes<CoefArgs>(
      cm_coef, kClassCoef, host, off, pl->dmem,
      [&](int k) {
        const Plan& p = geo[k].p;
        return CoefArgs{items[k].I_lo, items[k].p_lo, eps_dev + k, 1, p.c, p.h, p.w, p.coTR,
                        ws_rel<float>(geo[k].off_abar), ws_rel<float>(geo[k].off_bbar), 0,
                        p.wide_co && p.mean_ab ? ws_rel<float>(geo[k].off_x) : nullptr};
      },
      [](const Geo& g, int& nx, int& ny) {
        nx = g.p.co_nx;
        ny = g.p.co_ny;
      },
      [](const Geo& g) { return g.p.coLDS; }, geo, pl->launch.coef);
  build_classes<ApplyArgs>(
      cm_apply, kClassApply, host, off, pl->dmem,
      [&](int k) {
        const Plan& p = geo[k].p;
        return ApplyArgs{items[k].I_hi, items[k].q_hi, ws_rel<float>(geo[k].off_abar),
                         ws_rel<float>(geo[k].off_bbar), p.h, p.w, p.H, p.W, p.RB, p.nrb, p.nxv,
                         (long long)p.planes * p.nrb * p.nxv, 0};
      },
      [](const Geo& g, int& nx, int& ny) {
        nx = (int)g.t_apply;
        ny = 1;
      },
      nullptr, geo, pl->launch.apply);
  build_classes<BwdHiArgs>(
      cm_hi, kClassBwdHi, host, off, pl->dmem,
      [&](int k) {
        const Plan& p = geo[k].p;
        return BwdHiArgs{items[k].I_hi, items[k].dq_hi, items[k].dI_hi,
                         ws_rel<float>(geo[k].off_abar), ws_rel<float>(geo[k].off_u), p.h, p.w,
                         p.H, p.W, p.bh, p.tw, p.nby, p.nbx, p.hw, 0,
                         ws_rel<float>(geo[k].off_bbar), items[k].q_hi};
      },
      [](const Geo& g, int& nx, int& ny) {
        nx = g.p.nbx;
        ny = g.p.nby;
      },
      [](const Geo& g) { return g.p.hiLDS; }, geo, pl->launch.bwd_hi);
  build_classes<BwdLoArgs>(
      cm_lo, kClassBwdLo, host, off, pl->dmem,
      [&](int k) {
        const Plan& p = geo[k].p;
        return BwdLoArgs{items[k].I_lo, items[k].p_lo, eps_dev + k, 1, p.c,
                         ws_rel<float>(geo[k].off_u), p.ubh, p.tw, p.nby, p.nbx, p.h, p.w, p.loTR,
                         items[k].dI_lo, items[k].dp_lo, ws_rel<float>(geo[k].off_eps), p.lo_nx,
                         p.lo_ny, p.wide_lo ? ws_rel<float>(geo[k].off_x) : nullptr};
      },
      [](const Geo& g, int& nx, int& ny) {
        nx = g.p.lo_nx;
        ny = g.p.lo_ny;
      },
      [](const Geo& g) { return g.p.loLDS; }, geo, pl->launch.bwd_lo);

  EpsItem* eh = reinterpret_cast<EpsItem*>(host.data() + eps_items_off);
  int e = 0;
  for (int k = 0; k < count; ++k)
    if (items[k].deps) {
      const Plan& p = geo[k].p;
      eh[e++] = EpsItem{ws_rel<float>(geo[k].off_eps), (long long)p.planes * p.lo_nx * p.lo_ny,
                        items[k].deps};
    }
  pl->launch.eps_items = reinterpret_cast<const EpsItem*>(pl->dmem + eps_items_off);
  pl->launch.eps_count = n_eps;
  if (hipMemcpy(pl->dmem, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(pl->dmem);
    delete pl;
    return set_error(GF_ERR_HIP, "device table upload failed");
  }
  *out = pl;
  return GF_OK;
}

hipError_t enqueue(const gf_plan* pl, int mode, char* ws, hipStream_t s) {
  switch (pl->dtype) {
    case GF_F32: return launch_batched_f32(pl->launch, mode, ws, s);
    case GF_F16: return launch_batched_f16(pl->launch, mode, ws, s);
    case GF_BF16: return launch_batched_bf16(pl->launch, mode, ws, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace
}  // namespace gf

extern "C" {

int32_t gf_plan_create(const gf_item_t* items, int32_t count, gf_plan_t** plan) {
  gf::set_error(GF_OK, "");
  return gf::create(items, count, plan);
}

size_t gf_plan_workspace_size(const gf_plan_t* plan) { return plan ? plan->ws_bytes : 0; }

int32_t gf_batched(gf_plan_t* plan, int32_t mode, void* ws, size_t ws_bytes, void* stream) {
  gf::set_error(GF_OK, "");
  if (!plan) return gf::set_error(GF_ERR_INVALID_ARG, "plan is NULL");
  const int run = mode & (GF_RUN_FORWARD | GF_RUN_BACKWARD);
  if (run == 0 || (mode & ~(GF_RUN_FORWARD | GF_RUN_BACKWARD | GF_RUN_GRAPH)) != 0)
    return gf::set_error(GF_ERR_INVALID_ARG, "mode needs GF_RUN_FORWARD and/or GF_RUN_BACKWARD");
  if ((run & GF_RUN_FORWARD) && !plan->all_q)
    return gf::set_error(GF_ERR_INVALID_ARG, "forward needs q_hi on every item");
  if ((run & GF_RUN_BACKWARD) && !plan->all_dq)
    return gf::set_error(GF_ERR_INVALID_ARG, "backward needs dq_hi on every item");
  if (!ws || ws_bytes < plan->ws_bytes)
    return gf::set_error(GF_ERR_WORKSPACE, "workspace smaller than gf_plan_workspace_size = " +
                                               std::to_string(plan->ws_bytes));
  if (gf::misaligned(ws)) return gf::set_error(GF_ERR_INVALID_ARG, "workspace must be 16-byte aligned");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
    return gf::set_error(GF_ERR_INVALID_ARG, "current device is not the plan's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (!(mode & GF_RUN_GRAPH)) {
    const hipError_t e = gf::enqueue(plan, run, w, s);
    return e == hipSuccess ? GF_OK : gf::set_error(GF_ERR_HIP, hipGetErrorString(e));
  }
  for (auto& g : plan->graphs)
    if (g.mode == run && g.ws == ws) {
      const hipError_t e = hipGraphLaunch(g.exec, s);
      return e == hipSuccess ? GF_OK : gf::set_error(GF_ERR_HIP, hipGetErrorString(e));
    }
  // record the launches on a private stream (nothing executes while
  // capturing), instantiate, then launch on the caller's stream
  if (!plan->cap && hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking) != hipSuccess)
    return gf::set_error(GF_ERR_HIP, "capture stream creation failed");
  if (hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return gf::set_error(GF_ERR_HIP, "stream capture failed to begin");
  gf::prof_mute(true);
  const hipError_t le = gf::enqueue(plan, run, w, plan->cap);
  gf::prof_mute(false);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(plan->cap, &graph);
  if (le != hipSuccess || ce != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return gf::set_error(GF_ERR_HIP, hipGetErrorString(le != hipSuccess ? le : ce));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return gf::set_error(GF_ERR_HIP, hipGetErrorString(ie));
  plan->graphs.push_back({run, ws, exec});
  const hipError_t e = hipGraphLaunch(exec, s);
  return e == hipSuccess ? GF_OK : gf::set_error(GF_ERR_HIP, hipGetErrorString(e));
}

void gf_plan_destroy(gf_plan_t* plan) {
  if (!plan) return;
  for (auto& g : plan->graphs) (void)hipGraphExecDestroy(g.exec);
  if (plan->cap) (void)hipStreamDestroy(plan->cap);
  if (plan->dmem) (void)hipFree(plan->dmem);
  delete plan;
}

}  // extern "C"

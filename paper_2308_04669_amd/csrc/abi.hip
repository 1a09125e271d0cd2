// C-ABI entry points: argument validation, workspace planning and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "blob_layout.h"
#include "launch.h"
#include "nedf.h"
#include "runtime.h"

namespace nedf {

namespace {
thread_local std::string g_last_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int64_t ray_count(const nedf_rays* r) {
  if (!r) return -1;
  if (r->kind == 0) return int64_t(r->camera.width) * int64_t(r->camera.height);
  return r->n;
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
std::map<const void*, size_t> g_prof_open;  // stream -> index of the open record

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool prof_on() { return g_prof_on; }

void prof_mark(const char* name, void* stream, bool begin) {
  if (!g_prof_on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (begin) {
    ProfRec r{name, prof_event(), prof_event()};
    if (!r.a || !r.b) return;
    hipEventRecord(r.a, s);
    g_prof_open[stream] = g_prof_recs.size();
    g_prof_recs.push_back(r);
  } else {
    auto it = g_prof_open.find(stream);
    if (it == g_prof_open.end()) return;
    hipEventRecord(g_prof_recs[it->second].b, s);
    g_prof_open.erase(it);
  }
}

int32_t fail(int32_t code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

size_t ws_fixed_bytes(int64_t n_rays) {
  size_t off = 256;                                  // status block
  off = align256(off + sizeof(WsCounters));          // counters
  off = align256(off + size_t(n_rays) * 8);          // packed keys
  off = align256(off + size_t(n_rays) * 4);          // opacity bits
  return off;
}

WsLayout ws_layout(int64_t n_rays, size_t ws_bytes) {
  WsLayout l;
  l.counters = 256;
  l.keys = align256(l.counters + sizeof(WsCounters));
  l.opac = align256(l.keys + size_t(n_rays) * 8);
  l.pairs = align256(l.opac + size_t(n_rays) * 4);
  int64_t cap = ws_bytes > l.pairs ? int64_t((ws_bytes - l.pairs) / 8) : 0;
  if (cap > (int64_t(1) << 31) - 1) cap = (int64_t(1) << 31) - 1;
  l.capacity = cap;
  l.end = l.pairs + size_t(cap) * 8;
  return l;
}

namespace {

int32_t check_rays(const nedf_rays* rays, RaySrcHost& rs) {
  if (!rays) return fail(NEDF_ERR_NULL, "rays is NULL");
  std::memset(&rs, 0, sizeof(rs));
  rs.kind = rays->kind;
  if (rays->kind == 0) {
    const nedf_camera& c = rays->camera;
    if (c.width <= 0 || c.height <= 0) return fail(NEDF_ERR_SHAPE, "camera width/height must be positive");
    if (!(c.fov_y_deg > 0.0 && c.fov_y_deg < 180.0)) return fail(NEDF_ERR_SHAPE, "camera fov must be in (0, 180)");
    double f[3] = {c.at[0] - c.eye[0], c.at[1] - c.eye[1], c.at[2] - c.eye[2]};
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0.0)) return fail(NEDF_ERR_SHAPE, "camera eye equals at");
    for (double& v : f) v /= fl;
    double r[3] = {f[1] * c.up[2] - f[2] * c.up[1], f[2] * c.up[0] - f[0] * c.up[2], f[0] * c.up[1] - f[1] * c.up[0]};
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 0.0)) return fail(NEDF_ERR_SHAPE, "camera up is parallel to the view direction");
    for (double& v : r) v /= rl;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    const double th = std::tan(c.fov_y_deg * M_PI / 360.0);
    const double aspect = double(c.width) / double(c.height);
    for (int i = 0; i < 3; ++i) {
      rs.eye[i] = float(c.eye[i]);
      rs.fwd[i] = float(f[i]);
      rs.right[i] = float(r[i] * th * aspect);
      rs.up[i] = float(u[i] * th);
    }
    rs.width = c.width;
    rs.height = c.height;
    rs.n = int64_t(c.width) * c.height;
  } else if (rays->kind == 1) {
    if (rays->n < 0) return fail(NEDF_ERR_SHAPE, "ray count is negative");
    if (rays->n > 0 && (!rays->origins || !rays->dirs)) return fail(NEDF_ERR_NULL, "ray arrays are NULL");
    if (!aligned16(rays->origins) || !aligned16(rays->dirs)) return fail(NEDF_ERR_ALIGN, "ray arrays must be 16-byte aligned");
    rs.o = rays->origins;
    rs.d = rays->dirs;
    rs.n = rays->n;
  } else {
    return fail(NEDF_ERR_SHAPE, "rays.kind must be 0 (camera) or 1 (arrays)");
  }
  if (rs.n > (int64_t(1) << 31) - 1) return fail(NEDF_ERR_SHAPE, "too many rays (limit 2^31 - 1)");
  return NEDF_OK;
}

int32_t check_scene(const nedf_scene* sc) {
  if (!sc) return fail(NEDF_ERR_NULL, "scene is NULL");
  if (sc->n_objects < 1 || sc->n_objects > NEDF_MAX_OBJECTS)
    return fail(NEDF_ERR_SHAPE, "n_objects must be 1..32");
  if (!sc->objects) return fail(NEDF_ERR_NULL, "scene.objects is NULL");
  if (sc->n_inst < 1) return fail(NEDF_ERR_SHAPE, "n_inst must be >= 1");
  if (!sc->inst_object || !sc->inst_w2l) return fail(NEDF_ERR_NULL, "instance arrays are NULL");
  if (!aligned16(sc->inst_object) || !aligned16(sc->inst_w2l)) return fail(NEDF_ERR_ALIGN, "instance arrays must be 16-byte aligned");
  for (int i = 0; i < sc->n_objects; ++i) {
    const nedf_object& o = sc->objects[i];
    if (!(o.bound > 0.0f)) return fail(NEDF_ERR_SHAPE, "object bound must be positive");
    if (o.field < NEDF_FIELD_SPHERE || o.field > NEDF_FIELD_MLP) return fail(NEDF_ERR_SHAPE, "unknown object field");
    if (o.field == NEDF_FIELD_SPHERE && !(o.param[2] > 0.0f)) return fail(NEDF_ERR_SHAPE, "sphere width must be positive");
    if (o.field == NEDF_FIELD_MLP) {
      if (!o.density.blob) return fail(NEDF_ERR_NULL, "MLP object without a density blob");
      if (!aligned16(o.density.blob)) return fail(NEDF_ERR_ALIGN, "density blob must be 16-byte aligned");
      if (o.sigma_mode < NEDF_SIGMA_SOFTPLUS || o.sigma_mode > NEDF_SIGMA_SDF) return fail(NEDF_ERR_SHAPE, "unknown sigma mode");
      if (o.sigma_mode == NEDF_SIGMA_SDF && !(o.param[1] > 0.0f)) return fail(NEDF_ERR_SHAPE, "sdf width must be positive");
      if (o.density.shape.in_kind != NEDF_IN_XYZ || o.density.shape.n_out != 1)
        return fail(NEDF_ERR_SHAPE, "density network must take xyz and output one value");
    }
  }
  return NEDF_OK;
}

int32_t hip_fail(hipError_t e, const char* where) {
  return fail(NEDF_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace
}  // namespace nedf

using namespace nedf;

extern "C" const char* nedf_version(void) { return "nedf-mi355x 0.1.0 (gfx950)"; }

extern "C" const char* nedf_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* nedf_status_string(int32_t s) {
  switch (s) {
    case NEDF_OK: return "ok";
    case NEDF_ERR_NULL: return "null pointer";
    case NEDF_ERR_SHAPE: return "bad shape";
    case NEDF_ERR_DTYPE: return "bad dtype";
    case NEDF_ERR_ALIGN: return "misaligned pointer";
    case NEDF_ERR_WORKSPACE: return "workspace too small";
    case NEDF_ERR_CAPACITY: return "pair capacity exceeded";
    case NEDF_ERR_HIP: return "HIP runtime error";
    case NEDF_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

extern "C" int32_t nedf_compose_transforms(const double* inst_G, int32_t n, float* inst_w2l,
                                           nedf_stream_t stream) {
  if (n < 0) return fail(NEDF_ERR_SHAPE, "nedf_compose_transforms: n < 0");
  if (n == 0) return NEDF_OK;
  if (!inst_G || !inst_w2l) return fail(NEDF_ERR_NULL, "nedf_compose_transforms: NULL argument");
  if (!aligned16(inst_G) || !aligned16(inst_w2l)) return fail(NEDF_ERR_ALIGN, "nedf_compose_transforms: misaligned");
  hipError_t e = launch_compose_transforms(inst_G, n, inst_w2l, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_compose_transforms");
  return NEDF_OK;
}

extern "C" size_t nedf_workspace_size(int32_t op, const nedf_scene* scene, const nedf_rays* rays,
                                      int64_t pair_capacity) {
  const int64_t n = ray_count(rays);
  if (n < 0 || !scene) {
    set_error("nedf_workspace_size: NULL scene or rays");
    return 0;
  }
  (void)op;
  int64_t cap = pair_capacity > 0 ? pair_capacity : n * int64_t(scene->n_inst > 0 ? scene->n_inst : 1);
  if (cap > (int64_t(1) << 31) - 1) cap = (int64_t(1) << 31) - 1;
  return ws_fixed_bytes(n) + size_t(cap) * 8;
}

extern "C" int32_t nedf_check_status(const void* ws, nedf_stream_t stream) {
  if (!ws) return fail(NEDF_ERR_NULL, "nedf_check_status: ws is NULL");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_check_status");
  int32_t st = 0;
  e = hipMemcpy(&st, ws, sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "nedf_check_status");
  if (st != NEDF_OK) fail(st, "device status: pair list overflow");
  return st;
}

extern "C" int32_t nedf_march_depth(const nedf_scene* scene, const nedf_rays* rays,
                                    const nedf_march_opts* opts, float* depth, int32_t* id,
                                    float* opacity, void* ws, size_t ws_bytes, nedf_stream_t stream) {
  int32_t st = check_scene(scene);
  if (st) return st;
  MarchLaunch m;
  std::memset(&m, 0, sizeof(m));
  st = check_rays(rays, m.rays);
  if (st) return st;
  if (!opts) return fail(NEDF_ERR_NULL, "opts is NULL");
  if (opts->n_samples < 1 || opts->n_samples > 4096) return fail(NEDF_ERR_SHAPE, "n_samples must be 1..4096");
  if (!(opts->hit_threshold > 0.0f && opts->hit_threshold <= 1.0f)) return fail(NEDF_ERR_SHAPE, "hit_threshold must be in (0, 1]");
  if (!opts->clip_to_bound && !(opts->t_far > opts->t_near && opts->t_near >= 0.0f))
    return fail(NEDF_ERR_SHAPE, "need 0 <= t_near < t_far");
  if (opts->dtype != NEDF_F32 && opts->dtype != NEDF_BF16) return fail(NEDF_ERR_DTYPE, "march dtype must be F32 or BF16");
  const int64_t n = m.rays.n;
  if (n == 0) return NEDF_OK;
  if (!depth || !id || !ws) return fail(NEDF_ERR_NULL, "depth, id and ws are required");
  if (!aligned16(depth) || !aligned16(id) || !aligned16(ws) || (opacity && !aligned16(opacity)))
    return fail(NEDF_ERR_ALIGN, "output buffers must be 16-byte aligned");
  m.lay = ws_layout(n, ws_bytes);
  if (ws_bytes < ws_fixed_bytes(n) + 8) return fail(NEDF_ERR_WORKSPACE, "workspace smaller than nedf_workspace_size()");
  m.n_obj = scene->n_objects;
  m.n_inst = scene->n_inst;
  bool have_shape = false;
  for (int i = 0; i < scene->n_objects; ++i) {
    const nedf_object& o = scene->objects[i];
    ObjDesc& d = m.obj[i];
    d.field = o.field;
    d.sigma_mode = o.sigma_mode;
    d.bound = o.bound;
    for (int j = 0; j < 6; ++j) d.param[j] = o.param[j];
    d.blob = static_cast<const uint8_t*>(o.density.blob);
    d.nedf_blob = static_cast<const uint8_t*>(o.nedf.blob);
    if (o.field == NEDF_FIELD_MLP) {
      const nedf_mlp_shape& s = o.density.shape;
      if (o.density.dtype != opts->dtype) return fail(NEDF_ERR_DTYPE, "density blob dtype differs from opts.dtype");
      if (!march_mlp_supported(opts->dtype, s.width, s.n_hidden, s.enc_L))
        return fail(NEDF_ERR_UNSUPPORTED, "density network shape not instantiated (width 64/3 hidden/L6 or 256/8/L10)");
      if (have_shape && (s.width != m.mlp_width || s.n_hidden != m.mlp_hidden || s.enc_L != m.mlp_L))
        return fail(NEDF_ERR_UNSUPPORTED, "all MLP objects of one call must share a network shape");
      have_shape = true;
      m.mlp_width = s.width;
      m.mlp_hidden = s.n_hidden;
      m.mlp_L = s.enc_L;
    }
  }
  m.inst_object = scene->inst_object;
  m.inst_w2l = scene->inst_w2l;
  m.n_samples = opts->n_samples;
  m.clip = opts->clip_to_bound;
  m.t_near = opts->t_near;
  m.t_far = opts->t_far;
  m.hit_thr = opts->hit_threshold;
  m.dtype = opts->dtype;
  m.ws = static_cast<uint8_t*>(ws);
  m.depth = depth;
  m.id = id;
  m.opacity = opacity;
  hipError_t e = launch_march(m, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_march_depth");
  return NEDF_OK;
}

extern "C" int32_t nedf_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_recs) {
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  g_prof_open.clear();
  g_prof_on = on != 0;
  return NEDF_OK;
}

extern "C" int32_t nedf_profile_read(int32_t max_stages, char* names, double* total_ms, int32_t* counts,
                                     int32_t* n_stages) {
  if (!names || !total_ms || !counts || !n_stages) return fail(NEDF_ERR_NULL, "nedf_profile_read: NULL argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<std::string> order;
  std::map<std::string, std::pair<double, int>> agg;
  for (auto& r : g_prof_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(NEDF_ERR_HIP, "nedf_profile_read: event sync failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    std::string n(r.name);
    if (!agg.count(n)) order.push_back(n);
    agg[n].first += ms;
    agg[n].second += 1;
  }
  int32_t k = 0;
  for (auto& n : order) {
    if (k >= max_stages) break;
    std::strncpy(names + 64 * k, n.c_str(), 63);
    names[64 * k + 63] = 0;
    total_ms[k] = agg[n].first;
    counts[k] = agg[n].second;
    ++k;
  }
  *n_stages = k;
  return NEDF_OK;
}

extern "C" int32_t nedf_ws_counters(const void* ws, nedf_stream_t stream, int64_t* out2) {
  if (!ws || !out2) return fail(NEDF_ERR_NULL, "nedf_ws_counters: NULL argument");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nedf_ws_counters");
  WsCounters c;
  e = hipMemcpy(&c, static_cast<const uint8_t*>(ws) + 256, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "nedf_ws_counters");
  out2[0] = c.total_pairs;
  out2[1] = c.total_items;
  return NEDF_OK;
}

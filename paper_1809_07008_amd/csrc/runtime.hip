// runtime.hip -- host side of the C-ABI declared in include/imb.h: validation, device memory
// layout, kernel sequencing of the coupled step (Sec. 2.3: lattice step with the disks mapped
// onto the lattice, then forces, then DEM), readback, checkpoints and timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "runtime.h"

using namespace imb;

namespace imb {

static thread_local std::string g_create_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves the simulation's device memory out of one buffer (offsets only when base is null).
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

static size_t storage_bytes(int storage) {
  return storage == IMB_STORAGE_F64 ? 8 : (storage == IMB_STORAGE_F32 ? 4 : 2);
}

void sim_geometry(const imb_config& c, Geometry* g, int y0, int rows) {
  g->tw = c.tile_w ? c.tile_w : 64;
  g->rows = c.tile_rows ? c.tile_rows : 1;
  g->tw_log = 0;
  while ((1 << g->tw_log) < g->tw) g->tw_log++;
  g->th = (BLOCK >> g->tw_log) * g->rows;
  g->y0 = rows > 0 ? y0 : 0;
  g->nyl = rows > 0 ? rows : c.ny;
  g->yoff = rows > 0 ? g->y0 - 1 : 0;
  g->tiles_x = (c.nx + g->tw - 1) / g->tw;
  g->tiles_y = (g->nyl + g->th - 1) / g->th;
  g->tiles_yg = (c.ny + g->th - 1) / g->th;
  g->ty_off = g->y0 / g->th;
  g->pitch = (int)align_up((size_t)c.nx, 64);
  g->plane = (long long)g->pitch * (rows > 0 ? g->nyl + 2 : g->nyl);
}

size_t layout(const imb_config& c, char* base, DeviceLayout* L, int y0, int rows) {
  Geometry g;
  sim_geometry(c, &g, y0, rows);
  const size_t mp = (size_t)std::max(c.max_particles, 1);
  const size_t es = storage_bytes(c.storage);
  Carver cv{base};
  DeviceLayout d{};
  d.f[0] = cv.take<char>(NQ * (size_t)g.plane * es);
  d.f[1] = cv.take<char>(NQ * (size_t)g.plane * es);
  ParticleState& s = d.ps;
  s.x = cv.take<double>(mp); s.y = cv.take<double>(mp); s.r = cv.take<double>(mp);
  s.vx = cv.take<double>(mp); s.vy = cv.take<double>(mp); s.om = cv.take<double>(mp);
  s.mode = cv.take<int>(mp);
  s.fcx = cv.take<double>(mp); s.fcy = cv.take<double>(mp);
  s.tcz = cv.take<double>(mp);
  s.hid = cv.take<int>(mp * HK); s.hsp = cv.take<double>(mp * HK);
  s.hw = cv.take<double>(mp * 2);
  s.Fx = cv.take<double>(mp); s.Fy = cv.take<double>(mp); s.Tz = cv.take<double>(mp);
  s.xref = cv.take<double>(mp); s.yref = cv.take<double>(mp);
  s.nbr = cv.take<int>(mp * NBMAX);
  s.nnbr = cv.take<int>(mp);
  s.rebuild = cv.take<int>(1);
  for (int k = 0; k < 2; ++k) {  // tab[0] directly follows the particle state (see set_particles)
    d.tab[k].box = cv.take<int4>(mp);
    d.tab[k].pos = cv.take<double4>(mp);
    d.tab[k].vel = cv.take<double4>(mp);
    d.band_mask[k] = cv.take<unsigned long long>((size_t)MASK_WORDS * g.tiles_y);
  }
  d.err = cv.take<int>(1);
  d.J = cv.take<double>(1);
  d.w = cv.take<double>(3 * mp);
  d.seed = cv.take<unsigned>(2);
  d.force = cv.take<double4>(mp * DISK_PARTS);
  if (L) *L = d;
  return align_up(cv.off, 256);
}

int validate_config(const imb_config* c, std::string* why) {
  char buf[256];
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return IMB_EINVAL;
  };
  if (!c) return bad("null configuration");
  if (c->nx < 2 || c->ny < 2) return bad("nx and ny must be >= 2");
  if ((long long)c->nx * c->ny > (1ll << 31)) return bad("lattice too large");
  if (c->storage < IMB_STORAGE_F64 || c->storage > IMB_STORAGE_F16) return bad("unknown storage");
  if (!(c->tau0 > 0.5) || !std::isfinite(c->tau0)) return bad("tau0 must exceed 1/2");
  if (!(c->smag_cs >= 0.0)) return bad("Smagorinsky constant must be >= 0");
  if (c->eps_subcells < 0 || c->eps_subcells > 64) return bad("eps_subcells must be 0..64");
  if (c->reserved != 0) return bad("reserved must be 0");
  if (!(std::fabs(c->wall_ux_bottom) <= 0.3) || !(std::fabs(c->wall_ux_top) <= 0.3))
    return bad("wall velocities must be finite and at most 0.3 in magnitude");
  if (!(c->flags & IMB_FLAG_WALLS) && (c->wall_ux_bottom != 0.0 || c->wall_ux_top != 0.0))
    return bad("moving walls need walls");
  if (!(c->kt >= 0.0 && c->kt < 1e300) || !(c->mu >= 0.0 && c->mu < 1e300))
    return bad("kt and mu must be finite and >= 0");
  if (c->n_sub < 1 || c->n_sub > 100000) return bad("n_sub must be in 1..100000");
  if (c->contact_model != IMB_CONTACT_LINEAR && c->contact_model != IMB_CONTACT_HERTZ_MINDLIN)
    return bad("unknown contact_model");
  if (c->contact_model == IMB_CONTACT_HERTZ_MINDLIN &&
      (!(c->young > 0.0 && c->young < 1e300) || !(c->poisson >= 0.0 && c->poisson < 0.5)))
    return bad("Hertz-Mindlin needs young > 0 and 0 <= poisson < 0.5");
  if (c->reserved2 != 0) return bad("reserved2 must be 0");
  if (!(c->rho0 > 0.0)) return bad("rho0 must be positive");
  if (!(c->kn >= 0.0) || !(c->damping_ratio >= 0.0) || !(c->rho_solid > 0.0))
    return bad("DEM parameters out of range");
  if (!std::isfinite(c->gx) || !std::isfinite(c->gy)) return bad("body force must be finite");
  if (c->max_particles < 0 || c->max_particles > MAX_PARTICLES) {
    snprintf(buf, sizeof buf, "max_particles must be in 0..%d", MAX_PARTICLES);
    return bad(buf);
  }
  const int tw = c->tile_w ? c->tile_w : 64;
  if (tw != 16 && tw != 32 && tw != 64 && tw != 128 && tw != 256)
    return bad("tile_w must be 16, 32, 64, 128 or 256");
  const int rows = c->tile_rows ? c->tile_rows : 1;
  if (rows != 1 && rows != 2 && rows != 4) return bad("tile_rows must be 1, 2 or 4");
  if (c->flags & ~IMB_FLAG_WALLS) return bad("unknown flag");
  return IMB_OK;
}

int hip_fail(std::string* err, hipError_t e, const char* what) {
  if (err) *err = std::string(what) + ": " + hipGetErrorString(e);
  return IMB_EHIP;
}

int map_device_error(int bits) {
  if (bits & ERR_RHO) return IMB_EUNSTABLE;
  if (bits & (ERR_MOVE | ERR_LEFT)) return IMB_EDEM;
  if (bits) return IMB_EOVERFLOW;
  return IMB_OK;
}

std::string describe_device_error(int bits) {
  std::string s;
  if (bits & ERR_TILE_LIST) s += "more than 32 disk boxes touch one tile; ";
  if (bits & ERR_SLOTS) s += "a disk box spans more than 64 tiles; ";
  if (bits & ERR_CELL) s += "more than 4 disks cover one cell or one thread column; ";
  if (bits & ERR_RHO) s += "non-finite or non-positive density; ";
  if (bits & ERR_NBR) s += "DEM neighbour list overflow; ";
  if (bits & ERR_MOVE) s += "a disk moved more than one cell in one step; ";
  if (bits & ERR_LEFT) s += "a disk centre left the channel; ";
  if (bits & ERR_CONTACTS)
    s += "a disk touches more than " + std::to_string(HK) + " others at once; ";
  return s;
}

}  // namespace imb

// ======================================================================= imb_sim
struct imb_sim {
  imb_config cfg;
  imb_config layout_cfg;  // configuration the device memory was carved for
  hipStream_t stream = nullptr;
  char* mem = nullptr;
  size_t mem_bytes = 0;
  bool owns = false;
  Geometry g;
  DeviceLayout d;
  int cur = 0;  // buffer holding the stored state
  int np = 0;
  int64_t steps = 0;
  std::string err;
  double* stage = nullptr;  // readback staging (library-owned)
  size_t stage_bytes = 0;
  bool timing = false;
  std::vector<hipEvent_t> ev_k[2];  // start/stop pairs: lattice kernel, particle phase
  double k_ms[2] = {0, 0};
  int64_t k_n[2] = {0, 0};
  std::vector<hipEvent_t> ev_pool;
  AdjointState* adj = nullptr;
  // captured step chains: graph[len][start buffer]; len index 0 = 2 steps, 1 = GRAPH_LONG steps
  hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  bool use_graphs = true;
  int device = -1;  // the HIP device current at creation (its memory and stream live there)
  // a slab of a lattice split in y (window rows; 0 = the whole lattice) and whether its ghost
  // rows below and above hold a neighbouring slab's rows
  int win_y0 = 0, win_rows = 0;
  int ghost[2] = {0, 0};
  int dparts = 1;  // lattice-step workgroups per disk (2 for a slab)
};

static constexpr int GRAPH_LONG = 32;

namespace imb {

LatticeArgs lattice_args(imb_sim* s, const void* src, void* dst) {
  LatticeArgs a{};
  a.nx = s->cfg.nx; a.ny = s->cfg.ny; a.pitch = s->g.pitch;
  a.walls = (s->cfg.flags & IMB_FLAG_WALLS) ? 1 : 0;
  a.tiles_x = s->g.tiles_x; a.tiles_y = s->g.tiles_y;
  a.tw_log = s->g.tw_log; a.rows = s->g.rows; a.plane = s->g.plane;
  a.tau0 = s->cfg.tau0; a.cs = s->cfg.smag_cs; a.gx = s->cfg.gx; a.gy = s->cfg.gy;
  a.eps_sub = s->cfg.eps_subcells;
  a.walls_move = a.walls && (s->cfg.wall_ux_bottom != 0.0 || s->cfg.wall_ux_top != 0.0);
  const int wj[4] = {7, 8, 5, 6};  // diagonals into the bottom wall, then into the top wall
  for (int k = 0; k < 4; ++k) {  // 6 w_j rho0 (c_j . u_w), evaluated as the oracle does
    const double uw = k < 2 ? s->cfg.wall_ux_bottom : s->cfg.wall_ux_top;
    a.wall_c[k] = 6.0 * w_of(wj[k]) * s->cfg.rho0 * ((double)cx_of(wj[k]) * uw);
    a.wall_cf[k] = (float)a.wall_c[k];
  }
  a.rho0 = s->cfg.rho0;
  a.src = src; a.dst = dst;
  a.y0 = s->g.y0; a.nyl = s->g.nyl; a.yoff = s->g.yoff;
  a.ty_off = s->g.ty_off; a.tiles_yg = s->g.tiles_yg;
  a.ghost_lo = s->ghost[0]; a.ghost_hi = s->ghost[1];
  // the tables of the step reading this source (no source: those of the stored state)
  const int t = src ? (src == s->d.f[1] ? 1 : 0) : s->cur;
  a.np = s->np; a.tab = s->d.tab[t]; a.err = s->d.err;
  a.band_mask = s->d.band_mask[t];
  a.pstride = std::max(s->cfg.max_particles, 1);
  a.seed = s->d.seed;
  a.seed_slot = t;
  a.nbr = s->d.ps.nbr;
  a.nnbr = s->d.ps.nnbr;
  a.force = s->d.force;
  a.dparts = s->dparts;
  return a;
}

ParticleArgs particle_args(imb_sim* s, int out_slot) {
  ParticleArgs a{};
  a.np = s->np; a.nx = s->cfg.nx; a.ny = s->cfg.ny;
  a.walls = (s->cfg.flags & IMB_FLAG_WALLS) ? 1 : 0;
  a.n_sub = s->cfg.n_sub; a.kn = s->cfg.kn; a.zeta = s->cfg.damping_ratio;
  a.rho_s = s->cfg.rho_solid;
  a.kt = s->cfg.kt; a.mu = s->cfg.mu;
  a.hertz = s->cfg.contact_model == IMB_CONTACT_HERTZ_MINDLIN ? 1 : 0;
  if (a.hertz) {  // evaluated as the simplified Hertz-Mindlin law defines them
    const double E = s->cfg.young, nu = s->cfg.poisson;
    const double G = E / (2.0 * (1.0 + nu));
    a.es_pp = E / (2.0 * (1.0 - nu * nu));
    a.es_pw = E / (1.0 - nu * nu);
    a.gs_pp = G / (2.0 * (2.0 - nu));
    a.gs_pw = G / (2.0 - nu);
    a.hm_damp = 2.0 * sqrt(5.0 / 6.0) * s->cfg.damping_ratio;
  }
  a.uw_bot = s->cfg.wall_ux_bottom; a.uw_top = s->cfg.wall_ux_top;
  a.tiles_x = s->g.tiles_x; a.tiles_y = s->g.tiles_y; a.tw = s->g.tw; a.th = s->g.th;
  a.tiles_yg = s->g.tiles_yg; a.ty_off = s->g.ty_off;
  a.s = s->d.ps; a.tab = s->d.tab[out_slot]; a.err = s->d.err;
  a.band_mask = s->d.band_mask[out_slot];
  a.direct = s->d.force;
  a.dparts = s->dparts;
  a.build_lists = 1;
  return a;
}

static hipEvent_t take_event(imb_sim* s) {
  if (!s->ev_pool.empty()) {
    hipEvent_t e = s->ev_pool.back();
    s->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

// One coupled step: the lattice kernel (every cell, each disk's force and torque), then the
// particle phase (DEM and the next step's disk tables, written to the other table copy).
void enqueue_step(imb_sim* s, const double* wfx, const double* wfy, const double* wtz,
                  double* J) {
  const int c = s->cur;
  LatticeArgs la = lattice_args(s, s->d.f[c], s->d.f[c ^ 1]);
  // timing: events recorded by the launch itself at the kernel's start and end
  auto timed = [&](int k, auto&& launch) {
    if (!s->timing) {
      launch(nullptr, nullptr);
      return;
    }
    hipEvent_t e0 = take_event(s), e1 = take_event(s);
    launch(e0, e1);
    s->ev_k[k].push_back(e0);
    s->ev_k[k].push_back(e1);
  };
  timed(0, [&](hipEvent_t e0, hipEvent_t e1) {
    launch_lattice_step(s->cfg.storage, la, s->stream, e0, e1);
  });
  if (s->np > 0) {
    ParticleArgs pa = particle_args(s, c ^ 1);
    pa.do_finalize = 1; pa.do_dem = 1; pa.do_table = 1;
    pa.wfx = wfx; pa.wfy = wfy; pa.wtz = wtz; pa.J = J;
    timed(1, [&](hipEvent_t e0, hipEvent_t e1) { launch_particle_phase(pa, s->stream, e0, e1); });
  }
  s->cur ^= 1;
  s->steps++;
}

// The same step with the per-disk force and torque of the lattice kernel kept in `force`
// (capacity >= np) instead of the simulation's buffer, launched directly (no graph, no event).
static void enqueue_step_into(imb_sim* s, double4* force) {
  const int c = s->cur;
  LatticeArgs la = lattice_args(s, s->d.f[c], s->d.f[c ^ 1]);
  la.force = force;
  launch_lattice_step(s->cfg.storage, la, s->stream);
  if (s->np > 0) {
    ParticleArgs pa = particle_args(s, c ^ 1);
    pa.do_finalize = 1; pa.do_dem = 1; pa.do_table = 1;
    pa.direct = force;
    launch_particle_phase(pa, s->stream);
  }
  s->cur ^= 1;
  s->steps++;
}

int sync_and_check(imb_sim* s) {
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(&s->err, e, "hipStreamSynchronize");
  int bits = 0;
  e = hipMemcpy(&bits, s->d.err, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpy(error flags)");
  const int rc = map_device_error(bits);
  if (rc) s->err = "device reported: " + describe_device_error(bits);
  return rc;
}

static int ensure_stage(imb_sim* s, size_t bytes) {
  if (s->stage_bytes >= bytes) return IMB_OK;
  if (s->stage) hipFree(s->stage);
  s->stage = nullptr;
  s->stage_bytes = 0;
  hipError_t e = hipMalloc((void**)&s->stage, bytes);
  if (e != hipSuccess) {
    s->stage = nullptr;
    s->err = "cannot allocate readback staging";
    return IMB_ENOMEM;
  }
  s->stage_bytes = bytes;
  return IMB_OK;
}

static int launch_check(imb_sim* s, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(&s->err, e, what);
  return IMB_OK;
}

int reset_device_error(imb_sim* s) {
  launch_fill_zero(s->d.err, sizeof(int), s->stream);
  return launch_check(s, "reset error flags");
}

}  // namespace imb

namespace imb {

void drop_graphs(imb_sim* s) {
  for (auto& row : s->graph)
    for (auto& g : row)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// Captures `len` consecutive steps starting from buffer `start` into an executable graph
// (captured on a private stream: the caller's stream may be the legacy null stream).
static hipGraphExec_t capture_steps(imb_sim* s, int len, int start) {
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
  const hipStream_t saved = s->stream;
  const int saved_cur = s->cur;
  const int64_t saved_steps = s->steps;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    s->stream = cs;
    s->cur = start;
    for (int k = 0; k < len; ++k) enqueue_step(s, nullptr, nullptr, nullptr, nullptr);
    s->stream = saved;
    if (hipStreamEndCapture(cs, &g) == hipSuccess && g) {
      if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) ge = nullptr;
      hipGraphDestroy(g);
    }
  }
  s->stream = saved;
  s->cur = saved_cur;
  s->steps = saved_steps;
  hipStreamDestroy(cs);
  hipGetLastError();
  return ge;
}

}  // namespace imb

namespace imb {

int create_sim(const imb_config* cfg, const imb_config* layout_cfg, void* hip_stream,
               void* dev_buf, size_t dev_bytes, imb_sim** out, int win_y0, int win_rows) {
  if (!out) return IMB_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = validate_config(cfg, &why);
  if (rc) {
    g_create_error = why;
    return rc;
  }
  imb_sim* s = new (std::nothrow) imb_sim();
  if (!s) return IMB_ENOMEM;
  s->cfg = *cfg;
  if (!s->cfg.tile_w) s->cfg.tile_w = 64;
  if (!s->cfg.tile_rows) s->cfg.tile_rows = 1;
  s->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&s->device) != hipSuccess) {
    hipGetLastError();
    s->device = -1;
  }
  s->win_y0 = win_rows > 0 ? win_y0 : 0;
  s->win_rows = win_rows > 0 ? win_rows : 0;
  s->dparts = win_rows > 0 ? DISK_PARTS : 1;  // a slab's few disks: two workgroups each
  sim_geometry(s->cfg, &s->g, s->win_y0, s->win_rows);
  s->layout_cfg = *layout_cfg;
  if (!s->layout_cfg.tile_w) s->layout_cfg.tile_w = 64;
  if (!s->layout_cfg.tile_rows) s->layout_cfg.tile_rows = 1;
  const size_t need = layout(s->layout_cfg, nullptr, nullptr, s->win_y0, s->win_rows);
  if (dev_buf) {
    if (dev_bytes < need || ((uintptr_t)dev_buf & 255)) {
      g_create_error = "bound device buffer too small or not 256-byte aligned";
      imb_destroy(s);
      return IMB_ENOMEM;
    }
    s->mem = (char*)dev_buf;
    s->owns = false;
  } else {
    hipError_t e = hipMalloc((void**)&s->mem, need);
    if (e != hipSuccess) {
      g_create_error = std::string("hipMalloc: ") + hipGetErrorString(e);
      s->mem = nullptr;
      imb_destroy(s);
      return IMB_ENOMEM;
    }
    s->owns = true;
  }
  s->mem_bytes = need;
  layout(s->layout_cfg, s->mem, &s->d, s->win_y0, s->win_rows);
  launch_fill_zero(s->mem, need, s->stream);
  rc = imb_init_equilibrium(s, s->cfg.rho0, 0.0, 0.0);
  if (!rc) rc = sync_and_check(s);
  if (rc) {
    g_create_error = s->err;
    imb_destroy(s);
    return rc;
  }
  *out = s;
  return IMB_OK;
}

int tile_rows_capacity(const imb_sim* s) {
  Geometry g;
  sim_geometry(s->layout_cfg, &g, s->win_y0, s->win_rows);
  return g.tiles_y;
}

int create_window_sim(const imb_config* cfg, int y0, int rows, void* hip_stream, imb_sim** out) {
  return create_sim(cfg, cfg, hip_stream, nullptr, 0, out, y0, rows);
}

void set_window_ghosts(imb_sim* s, int below, int above) {
  s->ghost[0] = below ? 1 : 0;
  s->ghost[1] = above ? 1 : 0;
}

const char* create_error() { return g_create_error.c_str(); }

int set_tile_shape(imb_sim* s, int tile_w, int tile_rows) {
  if (s->win_rows) {
    s->err = "a slab's tile shape is fixed by its split";
    return IMB_EINVAL;
  }
  imb_config c = s->cfg;
  c.tile_w = tile_w;
  c.tile_rows = tile_rows;
  std::string why;
  if (validate_config(&c, &why)) {
    s->err = why;
    return IMB_EINVAL;
  }
  Geometry g;
  sim_geometry(c, &g);
  if (g.tiles_y > tile_rows_capacity(s)) {
    s->err = "tile shape needs more tile rows than the memory layout holds";
    return IMB_EINVAL;
  }
  hipStreamSynchronize(s->stream);
  drop_graphs(s);
  s->cfg = c;
  s->g = g;
  if (s->np > 0) {
    ParticleArgs pa = particle_args(s, s->cur);
    pa.do_table = 1;
    launch_particle_phase(pa, s->stream);
  }
  return launch_check(s, "set_tile_shape");
}

}  // namespace imb

// =================================================================== C-ABI
extern "C" {

void imb_config_default(imb_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->nx = 64; c->ny = 64; c->storage = IMB_STORAGE_F64; c->n_sub = 10;
  c->tau0 = 0.6; c->smag_cs = 0.0; c->gx = 0.0; c->gy = 0.0; c->rho0 = 1.0;
  c->kn = 1.0e3; c->damping_ratio = 0.1; c->rho_solid = 1.0; c->max_particles = 64;
  c->flags = IMB_FLAG_WALLS; c->tile_w = 64; c->tile_rows = 1;
  c->eps_subcells = 0; c->reserved = 0; c->wall_ux_bottom = 0.0; c->wall_ux_top = 0.0;
  c->kt = 0.0; c->mu = 0.0;
  c->contact_model = IMB_CONTACT_LINEAR; c->reserved2 = 0; c->young = 0.0; c->poisson = 0.0;
}

int imb_required_bytes(const imb_config* cfg, size_t* bytes) {
  if (!bytes) return IMB_EINVAL;
  int rc = validate_config(cfg, nullptr);
  if (rc) return rc;
  *bytes = layout(*cfg, nullptr, nullptr);
  return IMB_OK;
}

int imb_create(const imb_config* cfg, void* hip_stream, void* dev_buf, size_t dev_bytes,
               imb_sim** out) {
  return imb::create_sim(cfg, cfg, hip_stream, dev_buf, dev_bytes, out);
}

void imb_destroy(imb_sim* s) {
  if (!s) return;
  hipStreamSynchronize(s->stream);
  drop_graphs(s);
  free_adjoint(s);
  for (auto& v : s->ev_k)
    for (auto e : v) hipEventDestroy(e);
  for (auto e : s->ev_pool) hipEventDestroy(e);
  if (s->stage) hipFree(s->stage);
  if (s->owns && s->mem) hipFree(s->mem);
  delete s;
}

int imb_init_equilibrium(imb_sim* s, double rho, double ux, double uy) {
  if (!s) return IMB_EINVAL;
  if (!(rho > 0.0) || !std::isfinite(ux) || !std::isfinite(uy)) {
    s->err = "invalid equilibrium state";
    return IMB_EINVAL;
  }
  double feq[NQ];
  const double uu = ux * ux + uy * uy;
  for (int i = 0; i < NQ; ++i) {
    const double cu = (double)cx_of(i) * ux + (double)cy_of(i) * uy;
    feq[i] = w_of(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
  LatticeArgs a = lattice_args(s, nullptr, nullptr);
  launch_unstream(s->cfg.storage, a, nullptr, feq, s->d.f[s->cur], s->stream);
  return launch_check(s, "init_equilibrium");
}

int imb_set_populations(imb_sim* s, const double* host_f) {
  if (!s || !host_f) return IMB_EINVAL;
  const size_t n = (size_t)NQ * s->cfg.nx * s->cfg.ny;
  int rc = ensure_stage(s, n * sizeof(double));
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(s->stage, host_f, n * sizeof(double), hipMemcpyHostToDevice,
                                s->stream);
  if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
  LatticeArgs a = lattice_args(s, nullptr, nullptr);
  launch_unstream(s->cfg.storage, a, s->stage, nullptr, s->d.f[s->cur], s->stream);
  rc = launch_check(s, "set_populations");
  if (rc) return rc;
  return sync_and_check(s);
}

int imb_get_populations(imb_sim* s, double* host_f) {
  if (!s || !host_f) return IMB_EINVAL;
  const size_t n = (size_t)NQ * s->cfg.nx * s->cfg.ny;
  int rc = ensure_stage(s, n * sizeof(double));
  if (rc) return rc;
  LatticeArgs a = lattice_args(s, nullptr, nullptr);
  launch_gather(s->cfg.storage, a, s->d.f[s->cur], s->stage, nullptr, nullptr, nullptr,
                s->stream);
  rc = launch_check(s, "get_populations");
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(host_f, s->stage, n * sizeof(double), hipMemcpyDeviceToHost,
                                s->stream);
  if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
  return sync_and_check(s);
}

int imb_get_fields(imb_sim* s, double* rho, double* ux, double* uy) {
  if (!s) return IMB_EINVAL;
  const size_t n = (size_t)s->cfg.nx * s->cfg.ny;
  int rc = ensure_stage(s, 3 * n * sizeof(double));
  if (rc) return rc;
  LatticeArgs a = lattice_args(s, nullptr, nullptr);
  launch_gather(s->cfg.storage, a, s->d.f[s->cur], nullptr, s->stage, s->stage + n,
                s->stage + 2 * n, s->stream);
  rc = launch_check(s, "get_fields");
  if (rc) return rc;
  double* outs[3] = {rho, ux, uy};
  for (int k = 0; k < 3; ++k) {
    if (!outs[k]) continue;
    hipError_t e = hipMemcpyAsync(outs[k], s->stage + k * n, n * sizeof(double),
                                  hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
  }
  return sync_and_check(s);
}

int imb_get_solid_field(imb_sim* s, double* host_eps) {
  if (!s || !host_eps) return IMB_EINVAL;
  const size_t n = (size_t)s->cfg.nx * s->cfg.ny;
  int rc = ensure_stage(s, n * sizeof(double));
  if (rc) return rc;
  LatticeArgs a = lattice_args(s, nullptr, nullptr);
  launch_solid_field(s->cfg.storage, a, s->stage, s->stream);
  rc = launch_check(s, "get_solid_field");
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(host_eps, s->stage, n * sizeof(double), hipMemcpyDeviceToHost,
                                s->stream);
  if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
  return sync_and_check(s);
}

int imb_set_particles(imb_sim* s, int32_t n, const double* x, const double* y, const double* r,
                      const double* vx, const double* vy, const double* om,
                      const int32_t* mode) {
  if (!s) return IMB_EINVAL;
  if (n < 0 || n > s->cfg.max_particles) {
    s->err = "particle count exceeds max_particles";
    return IMB_EINVAL;
  }
  if (n > 0 && (!x || !y || !r || !vx || !vy || !om || !mode)) {
    s->err = "null particle array";
    return IMB_EINVAL;
  }
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const bool walls = s->cfg.flags & IMB_FLAG_WALLS;
  for (int p = 0; p < n; ++p) {
    char buf[200];
    bool ok = r[p] > 0.0 && 2.0 * (r[p] + 2.0) < nx && 2.0 * (r[p] + 2.0) < ny &&
              x[p] >= 0.0 && x[p] < nx && std::isfinite(y[p]) && std::isfinite(vx[p]) &&
              std::isfinite(vy[p]) && std::isfinite(om[p]) && mode[p] >= 0 && mode[p] <= 2;
    if (ok && walls) ok = y[p] >= -0.5 && y[p] <= ny - 0.5;
    if (ok && !walls) ok = y[p] >= 0.0 && y[p] < ny;
    int4 b;
    if (ok && !tile_box(x[p], y[p], r[p], nx, ny, walls, s->g.tiles_x, s->g.tiles_yg, s->g.tw,
                        s->g.th, &b)) {
      snprintf(buf, sizeof buf, "disk %d spans more than %d tiles", p, MAXSLOT);
      s->err = buf;
      return IMB_EINVAL;
    }
    if (!ok) {
      snprintf(buf, sizeof buf, "disk %d out of range (need r > 0, 2(r+2) < min(nx,ny), "
               "0 <= x < nx, centre inside the channel, mode 0..2)", p);
      s->err = buf;
      return IMB_EINVAL;
    }
  }
  hipStreamSynchronize(s->stream);
  drop_graphs(s);
  disarm_adjoint(s);
  s->np = n;
  ParticleState& ps = s->d.ps;
  const size_t mp = (size_t)std::max(s->cfg.max_particles, 1);
  // zero every per-particle array first (DEM caches, forces, lists)
  launch_fill_zero(ps.x, (char*)(s->d.tab[0].box) - (char*)ps.x, s->stream);
  (void)mp;
  if (n > 0) {
    const double* src[6] = {x, y, r, vx, vy, om};
    double* dst[6] = {ps.x, ps.y, ps.r, ps.vx, ps.vy, ps.om};
    for (int k = 0; k < 6; ++k) {
      hipError_t e = hipMemcpyAsync(dst[k], src[k], n * sizeof(double), hipMemcpyHostToDevice,
                                    s->stream);
      if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
    }
    hipError_t e = hipMemcpyAsync(ps.mode, mode, n * sizeof(int), hipMemcpyHostToDevice,
                                  s->stream);
    if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
    e = hipMemcpyAsync(ps.xref, x, n * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ps.yref, y, n * sizeof(double), hipMemcpyHostToDevice, s->stream);
    const int one = 1;
    if (e == hipSuccess)
      e = hipMemcpyAsync(ps.rebuild, &one, sizeof(int), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
    ParticleArgs pa = particle_args(s, s->cur);
    pa.init_contacts = 1;
    pa.do_table = 1;
    launch_particle_phase(pa, s->stream);
    int rc = launch_check(s, "set_particles");
    if (rc) return rc;
  }
  int rc = reset_device_error(s);
  if (rc) return rc;
  hipStreamSynchronize(s->stream);
  return sync_and_check(s);
}

int imb_step(imb_sim* s, int32_t nsteps) {
  if (!s || nsteps < 0) return IMB_EINVAL;
  // per-kernel event timing needs the individual launches
  if (!s->use_graphs || s->timing) {
    for (int k = 0; k < nsteps; ++k) enqueue_step(s, nullptr, nullptr, nullptr, nullptr);
    return launch_check(s, "step");
  }
  while (nsteps > 0) {
    const int li = nsteps >= GRAPH_LONG ? 1 : (nsteps >= 2 ? 0 : -1);
    if (li < 0) {
      enqueue_step(s, nullptr, nullptr, nullptr, nullptr);
      --nsteps;
      continue;
    }
    const int len = li ? GRAPH_LONG : 2;
    hipGraphExec_t& ge = s->graph[li][s->cur];
    if (!ge) ge = capture_steps(s, len, s->cur);
    if (!ge) {  // capture unsupported: plain launches
      s->use_graphs = false;
      for (int k = 0; k < nsteps; ++k) enqueue_step(s, nullptr, nullptr, nullptr, nullptr);
      return launch_check(s, "step");
    }
    hipError_t e = hipGraphLaunch(ge, s->stream);
    if (e != hipSuccess) return hip_fail(&s->err, e, "hipGraphLaunch");
    s->steps += len;  // an even number of steps leaves the buffer parity unchanged
    nsteps -= len;
  }
  return launch_check(s, "step");
}

int imb_set_graphs(imb_sim* s, int enable) {
  if (!s) return IMB_EINVAL;
  hipStreamSynchronize(s->stream);
  drop_graphs(s);
  s->use_graphs = enable != 0;
  return IMB_OK;
}

// ------------------------------------------------------- stepping without allocation
// imb_step_noalloc keeps the per-disk force and torque that the lattice kernel hands to the
// particle phase in this file-scope device array (one copy on every GPU the library runs on,
// held until the process ends) instead of in the simulation's buffer.  Host code never passes
// the array's name to a kernel: its device address is resolved once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
static constexpr int NOALLOC_MAX_DISKS = 8192;  // one share per disk: 256 KiB
static constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) double4 scratch[NOALLOC_MAX_DISKS];
static std::mutex g_scratch_mu;
static double4* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int imb_step_noalloc(imb_sim* s, int32_t nsteps) {
  if (!s || nsteps < 0) return IMB_EINVAL;
  if (s->np * s->dparts > NOALLOC_MAX_DISKS) {
    s->err = "imb_step_noalloc: more disks than its scratch holds (8192)";
    return IMB_EINVAL;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return hip_fail(&s->err, hipGetLastError(), "hipGetDevice");
  if (dev != s->device || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    s->err = "imb_step_noalloc: the current device is not the one the simulation was created on";
    return IMB_EINVAL;
  }
  double4* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return hip_fail(&s->err, e, "hipGetSymbolAddress(scratch)");
      g_scratch_ptr[dev] = (double4*)p;
    }
    ptr = g_scratch_ptr[dev];
  }
  for (int k = 0; k < nsteps; ++k) enqueue_step_into(s, ptr);
  return launch_check(s, "step_noalloc");
}

int imb_prepare_graphs(imb_sim* s) {
  if (!s) return IMB_EINVAL;
  hipStreamSynchronize(s->stream);
  if (!s->use_graphs) return IMB_OK;
  for (int li = 0; li < 2; ++li)
    for (int start = 0; start < 2; ++start) {
      hipGraphExec_t& ge = s->graph[li][start];
      if (!ge) ge = capture_steps(s, li ? GRAPH_LONG : 2, start);
      if (!ge) {  // capture unsupported: imb_step launches directly
        s->use_graphs = false;
        return IMB_OK;
      }
      if (hipGraphUpload(ge, s->stream) != hipSuccess) hipGetLastError();
    }
  return sync_and_check(s);
}

int imb_get_forces(imb_sim* s, double* fx, double* fy, double* tz) {
  if (!s) return IMB_EINVAL;
  const size_t n = (size_t)s->np;
  double* outs[3] = {fx, fy, tz};
  const double* srcs[3] = {s->d.ps.Fx, s->d.ps.Fy, s->d.ps.Tz};
  for (int k = 0; k < 3 && n; ++k) {
    if (!outs[k]) continue;
    hipError_t e = hipMemcpyAsync(outs[k], srcs[k], n * sizeof(double), hipMemcpyDeviceToHost,
                                  s->stream);
    if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
  }
  return sync_and_check(s);
}

int imb_get_particles(imb_sim* s, double* x, double* y, double* vx, double* vy, double* om) {
  if (!s) return IMB_EINVAL;
  const size_t n = (size_t)s->np;
  double* outs[5] = {x, y, vx, vy, om};
  const double* srcs[5] = {s->d.ps.x, s->d.ps.y, s->d.ps.vx, s->d.ps.vy, s->d.ps.om};
  for (int k = 0; k < 5 && n; ++k) {
    if (!outs[k]) continue;
    hipError_t e = hipMemcpyAsync(outs[k], srcs[k], n * sizeof(double), hipMemcpyDeviceToHost,
                                  s->stream);
    if (e != hipSuccess) return hip_fail(&s->err, e, "hipMemcpyAsync");
  }
  return sync_and_check(s);
}

int imb_get_counts(imb_sim* s, int32_t* n_particles, int64_t* steps) {
  if (!s) return IMB_EINVAL;
  if (n_particles) *n_particles = s->np;
  if (steps) *steps = s->steps;
  return IMB_OK;
}

int imb_sync(imb_sim* s) {
  if (!s) return IMB_EINVAL;
  return sync_and_check(s);
}

// ----------------------------------------------------------------------- checkpoints
namespace {
struct StateHeader {
  char magic[8];
  imb_config cfg;
  int32_t np;
  uint32_t seed;  // stochastic-rounding step counter of the stored state
  int64_t steps;
  uint64_t pop_bytes;
};
}  // namespace

// per disk in a checkpoint: 11 FP64 values and the mode, the contact torque, the two wall
// springs, and the HK tangential springs with their partners
constexpr size_t PARTICLE_STATE_BYTES =
    11 * sizeof(double) + sizeof(int) + (3 + HK) * sizeof(double) + HK * sizeof(int);

static size_t state_bytes(imb_sim* s) {
  const size_t pop = NQ * (size_t)s->g.plane * storage_bytes(s->cfg.storage);
  const size_t npb = (size_t)s->np;
  return sizeof(StateHeader) + pop + npb * PARTICLE_STATE_BYTES;
}

int imb_state_bytes(imb_sim* s, size_t* bytes) {
  if (!s || !bytes) return IMB_EINVAL;
  *bytes = state_bytes(s);
  return IMB_OK;
}

int imb_save_state(imb_sim* s, void* host_buf, size_t bytes) {
  if (!s || !host_buf) return IMB_EINVAL;
  if (bytes < state_bytes(s)) {
    s->err = "checkpoint buffer too small";
    return IMB_EINVAL;
  }
  StateHeader h{};
  std::memcpy(h.magic, "IMBSTAT1", 8);
  h.cfg = s->cfg;
  h.np = s->np;
  h.steps = s->steps;
  h.pop_bytes = NQ * (size_t)s->g.plane * storage_bytes(s->cfg.storage);
  hipStreamSynchronize(s->stream);
  if (hipMemcpy(&h.seed, s->d.seed + s->cur, sizeof(unsigned), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return hip_fail(&s->err, hipGetLastError(), "save_state seed");
  char* out = (char*)host_buf;
  std::memcpy(out, &h, sizeof h);
  out += sizeof h;
  hipError_t e = hipMemcpyAsync(out, s->d.f[s->cur], h.pop_bytes, hipMemcpyDeviceToHost,
                                s->stream);
  out += h.pop_bytes;
  const ParticleState& ps = s->d.ps;
  const double* arrs[11] = {ps.x, ps.y, ps.r, ps.vx, ps.vy, ps.om,
                            ps.fcx, ps.fcy, ps.Fx, ps.Fy, ps.Tz};
  for (int k = 0; k < 11 && e == hipSuccess && s->np; ++k) {
    e = hipMemcpyAsync(out, arrs[k], s->np * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    out += s->np * sizeof(double);
  }
  if (e == hipSuccess && s->np) {
    e = hipMemcpyAsync(out, ps.mode, s->np * sizeof(int), hipMemcpyDeviceToHost, s->stream);
    out += s->np * sizeof(int);
  }
  // the contact torque and the tangential springs
  const std::pair<const void*, size_t> extra[4] = {
      {ps.tcz, s->np * sizeof(double)}, {ps.hw, 2 * s->np * sizeof(double)},
      {ps.hsp, HK * s->np * sizeof(double)}, {ps.hid, HK * s->np * sizeof(int)}};
  for (int k = 0; k < 4 && e == hipSuccess && s->np; ++k) {
    e = hipMemcpyAsync(out, extra[k].first, extra[k].second, hipMemcpyDeviceToHost, s->stream);
    out += extra[k].second;
  }
  if (e != hipSuccess) return hip_fail(&s->err, e, "save_state copy");
  return sync_and_check(s);
}

int imb_load_state(imb_sim* s, const void* host_buf, size_t bytes) {
  if (!s || !host_buf || bytes < sizeof(StateHeader)) return IMB_EINVAL;
  StateHeader h;
  std::memcpy(&h, host_buf, sizeof h);
  if (std::memcmp(h.magic, "IMBSTAT1", 8) != 0) {
    s->err = "not a checkpoint";
    return IMB_EINVAL;
  }
  imb_config a = h.cfg, b = s->cfg;
  if (std::memcmp(&a, &b, sizeof a) != 0 || h.np > s->cfg.max_particles || h.np < 0) {
    s->err = "checkpoint configuration differs from this simulation";
    return IMB_EINVAL;
  }
  const size_t pop = NQ * (size_t)s->g.plane * storage_bytes(s->cfg.storage);
  const size_t need = sizeof h + pop + (size_t)h.np * PARTICLE_STATE_BYTES;
  if (bytes < need || h.pop_bytes != pop) {
    s->err = "checkpoint truncated";
    return IMB_EINVAL;
  }
  const char* in = (const char*)host_buf + sizeof h;
  hipStreamSynchronize(s->stream);
  drop_graphs(s);
  disarm_adjoint(s);
  s->cur = 0;
  s->np = h.np;
  s->steps = h.steps;
  ParticleState& ps = s->d.ps;
  launch_fill_zero(ps.x, (char*)(s->d.tab[0].box) - (char*)ps.x, s->stream);
  hipError_t e = hipMemcpyAsync(s->d.f[0], in, pop, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpy(s->d.seed, &h.seed, sizeof(unsigned), hipMemcpyHostToDevice);
  in += pop;
  double* arrs[11] = {ps.x, ps.y, ps.r, ps.vx, ps.vy, ps.om, ps.fcx, ps.fcy, ps.Fx, ps.Fy, ps.Tz};
  for (int k = 0; k < 11 && e == hipSuccess && s->np; ++k) {
    e = hipMemcpyAsync(arrs[k], in, s->np * sizeof(double), hipMemcpyHostToDevice, s->stream);
    in += s->np * sizeof(double);
  }
  if (e == hipSuccess && s->np) {
    e = hipMemcpyAsync(ps.mode, in, s->np * sizeof(int), hipMemcpyHostToDevice, s->stream);
    in += s->np * sizeof(int);
    const std::pair<void*, size_t> extra[4] = {
        {ps.tcz, s->np * sizeof(double)}, {ps.hw, 2 * s->np * sizeof(double)},
        {ps.hsp, HK * s->np * sizeof(double)}, {ps.hid, HK * s->np * sizeof(int)}};
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
      e = hipMemcpyAsync(extra[k].first, in, extra[k].second, hipMemcpyHostToDevice, s->stream);
      in += extra[k].second;
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(ps.xref, ps.x, s->np * sizeof(double), hipMemcpyDeviceToDevice,
                         s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ps.yref, ps.y, s->np * sizeof(double), hipMemcpyDeviceToDevice,
                         s->stream);
    const int one = 1;
    if (e == hipSuccess)
      e = hipMemcpyAsync(ps.rebuild, &one, sizeof(int), hipMemcpyHostToDevice, s->stream);
  }
  if (e != hipSuccess) return hip_fail(&s->err, e, "load_state copy");
  if (s->np) {
    ParticleArgs pa = particle_args(s, s->cur);
    pa.do_table = 1;
    launch_particle_phase(pa, s->stream);
  }
  int rc = reset_device_error(s);
  if (rc) return rc;
  hipStreamSynchronize(s->stream);
  return sync_and_check(s);
}

// --------------------------------------------------------------------------- timing
int imb_set_kernel_timing(imb_sim* s, int enable) {
  if (!s) return IMB_EINVAL;
  hipStreamSynchronize(s->stream);
  for (int k = 0; k < 2; ++k) {
    for (auto e : s->ev_k[k]) s->ev_pool.push_back(e);
    s->ev_k[k].clear();
    s->k_ms[k] = 0;
    s->k_n[k] = 0;
  }
  s->timing = enable != 0;
  return IMB_OK;
}

int imb_get_kernel_timing(imb_sim* s, double* lat_ms, int64_t* lat_n, double* par_ms,
                          int64_t* par_n) {
  if (!s) return IMB_EINVAL;
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(&s->err, e, "hipStreamSynchronize");
  for (int k = 0; k < 2; ++k) {
    std::vector<hipEvent_t>& v = s->ev_k[k];
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
      float t = 0;
      hipEventElapsedTime(&t, v[i], v[i + 1]);
      s->k_ms[k] += t;
      s->k_n[k] += 1;
      s->ev_pool.push_back(v[i]);
      s->ev_pool.push_back(v[i + 1]);
    }
    v.clear();
  }
  if (lat_ms) *lat_ms = s->k_ms[0];
  if (lat_n) *lat_n = s->k_n[0];
  if (par_ms) *par_ms = s->k_ms[1];
  if (par_n) *par_n = s->k_n[1];
  return IMB_OK;
}

int imb_copy_kernel(void* dst, const void* src, size_t n_bytes, void* stream) {
  if ((!dst || !src) && n_bytes) return IMB_EINVAL;
  if (((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) return IMB_EINVAL;
  if (n_bytes == 0) return IMB_OK;
  launch_copy(dst, src, n_bytes, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? IMB_OK : IMB_EHIP;
}

const char* imb_strerror(int code) {
  switch (code) {
    case IMB_OK: return "ok";
    case IMB_EINVAL: return "invalid argument";
    case IMB_ENOMEM: return "out of device memory";
    case IMB_EHIP: return "HIP runtime error";
    case IMB_EOVERFLOW: return "fixed-capacity list overflow";
    case IMB_EUNSTABLE: return "numerical instability (density)";
    case IMB_EDEM: return "DEM step out of range";
    case IMB_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
  }
}

const char* imb_last_error(const imb_sim* s) {
  return s ? s->err.c_str() : g_create_error.c_str();
}

const char* imb_version(void) { return "imb 0.1 (gfx950)"; }

}  // extern "C"

// ------------------------------------------------------------- internal accessors
namespace imb {
SimView sim_view(imb_sim* s) {
  SimView v;
  v.cfg = &s->cfg;
  v.g = &s->g;
  v.d = &s->d;
  v.stream = s->stream;
  v.cur = &s->cur;
  v.np = &s->np;
  v.steps = &s->steps;
  v.err = &s->err;
  v.adj = &s->adj;
  v.timing = &s->timing;
  return v;
}
}  // namespace imb

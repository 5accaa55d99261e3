// slab.hip -- one GPU's share of a lattice split into slabs of rows (y), and the driver that runs
// every slab of such a split on one device.
//
// Each slab ("rank") is a simulation that updates only its rows [y0, y0 + rows) and runs the
// same lattice kernel as the whole lattice (step.hip, its window instantiation).  Its population
// planes hold one ghost row on each side.  Streaming across a slab face needs the three
// populations that cross it (c_y = +1 upwards, -1 downwards); between steps they are copied
// from the neighbour's boundary row into the ghost row, plane by plane.  In the structure-of-
// arrays layout each of these is one contiguous row of nx elements, so nothing is packed and
// the lattice kernel reads a ghost row like any other.  A disk whose box meets several slabs is
// evaluated by each of them over its own rows; each slab writes its share of every disk's force
// and torque (zero for the disks that miss it).  The particle phase is replicated: every slab
// integrates the same disks from the same summed forces, and writes the disk tables and band
// lists of its own rows.
//
// Between the lattice kernels and the particle phases one kernel stands in for the two
// collectives of a multi-GPU run: it copies every crossing row into the neighbour's ghost row
// (the transfer over the inter-GPU links) and sums the per-slab force shares in slab order (the
// all-reduce).
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "runtime.h"

namespace imb {

constexpr int MAX_SLABS = 16;
constexpr int SLAB_GRAPH_LONG = 32;
constexpr int COPIES_PER_SLAB = 6;  // three crossing populations on each face

struct RowCopy {
  const void* from;
  void* to;
};

struct ExchangeArgs {
  const RowCopy* copy;             // [ncopy] rows of `words` 32-bit words (16-bit: half_words)
  int ncopy, words, half_words;
  int nslab, np;
  const double4* part[MAX_SLABS];  // each slab's shares of the per-disk force and torque
  double4* sum;                    // [np][DISK_PARTS]: their sum in slab order, in the first
};

// Grid: x over the words of a row, y over the copies; the extra row y = ncopy sums the forces.
__global__ __launch_bounds__(256) void k_exchange(ExchangeArgs a) {
  const int c = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  if (c < a.ncopy) {
    const RowCopy rc = a.copy[c];
    if (a.half_words) {
      for (int w = t; w < a.words; w += stride)
        ((unsigned short*)rc.to)[w] = ((const unsigned short*)rc.from)[w];
    } else {
      for (int w = t; w < a.words; w += stride) ((unsigned*)rc.to)[w] = ((const unsigned*)rc.from)[w];
    }
    return;
  }
  static_assert(DISK_PARTS == 2, "a slab's disks have two shares each");
  auto share = [&](int r, int p) {  // slab r's share: its two workgroups' parts added
    const double4 u = a.part[r][DISK_PARTS * p], v = a.part[r][DISK_PARTS * p + 1];
    return make_double4(u.x + v.x, u.y + v.y, u.z + v.z, 0.0);
  };
  for (int p = t; p < a.np; p += stride) {
    double4 s = share(0, p);
    for (int r = 1; r < a.nslab; ++r) {
      const double4 v = share(r, p);
      s.x += v.x;
      s.y += v.y;
      s.z += v.z;
    }
    a.sum[DISK_PARTS * p] = s;  // the particle phase adds the second slot, zero
    a.sum[DISK_PARTS * p + 1] = make_double4(0.0, 0.0, 0.0, 0.0);
  }
}

}  // namespace imb

using namespace imb;

struct imb_slab {
  imb_config cfg;
  int n = 0;                    // slabs
  std::vector<imb_sim*> rank;
  std::vector<SimView> view;
  int y0[MAX_SLABS] = {}, rows[MAX_SLABS] = {};
  hipStream_t stream = nullptr;
  char* xmem = nullptr;         // the row-copy tables and the summed forces
  double4* fsum = nullptr;
  ExchangeArgs xa[2] = {};      // exchange after a step that wrote population buffer k
  int xgrid = 1;
  double* stage = nullptr;
  size_t stage_bytes = 0;
  int np = 0;
  int64_t steps = 0;
  std::string err;
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  // per timed launch: (kind, slab, start, stop); kind 0 lattice, 1 exchange, 2 particle phase
  struct Timed {
    int kind, slab;
    hipEvent_t e0, e1;
  };
  std::vector<Timed> timed;
  double lat_ms[MAX_SLABS] = {}, par_ms[MAX_SLABS] = {}, xch_ms = 0.0;
  int64_t timed_steps = 0;
  hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
};

namespace {

thread_local std::string g_slab_create_error;

int slab_fail(imb_slab* S, hipError_t e, const char* what) {
  S->err = std::string(what) + ": " + hipGetErrorString(e);
  return IMB_EHIP;
}

hipEvent_t slab_event(imb_slab* S) {
  if (!S->ev_pool.empty()) {
    hipEvent_t e = S->ev_pool.back();
    S->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

void drop_slab_graphs(imb_slab* S) {
  for (auto& row : S->graph)
    for (auto& g : row)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// One coupled step of every slab on `st`: the slabs' lattice kernels, the exchange, then the
// slabs' particle phases (DEM from the summed forces; each slab's tables for the next step).
void enqueue_slab_step(imb_slab* S, hipStream_t st) {
  const int c = *S->view[0].cur;
  auto run = [&](int kind, int r, auto&& launch) {
    if (!S->timing) {
      launch(nullptr, nullptr);
      return;
    }
    hipEvent_t e0 = slab_event(S), e1 = slab_event(S);
    launch(e0, e1);
    S->timed.push_back({kind, r, e0, e1});
  };
  for (int r = 0; r < S->n; ++r) {
    LatticeArgs la = lattice_args(S->rank[r], S->view[r].d->f[c], S->view[r].d->f[c ^ 1]);
    run(0, r, [&](hipEvent_t e0, hipEvent_t e1) {
      launch_lattice_step(S->cfg.storage, la, st, e0, e1);
    });
  }
  const ExchangeArgs& xa = S->xa[c ^ 1];
  run(1, 0, [&](hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid(S->xgrid, xa.ncopy + 1);
    if (e0 || e1)
      hipExtLaunchKernelGGL(k_exchange, grid, dim3(256), 0, st, e0, e1, 0, xa);
    else
      hipLaunchKernelGGL(k_exchange, grid, dim3(256), 0, st, xa);
  });
  if (S->np > 0)
    for (int r = 0; r < S->n; ++r) {
      ParticleArgs pa = particle_args(S->rank[r], c ^ 1);
      pa.do_finalize = 1; pa.do_dem = 1; pa.do_table = 1;
      pa.direct = S->fsum;
      run(2, r, [&](hipEvent_t e0, hipEvent_t e1) { launch_particle_phase(pa, st, e0, e1); });
    }
  for (int r = 0; r < S->n; ++r) {
    *S->view[r].cur ^= 1;
    (*S->view[r].steps)++;
  }
  S->steps++;
}

hipGraphExec_t capture_slab_steps(imb_slab* S, int len, int start) {
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
  std::vector<int> cur(S->n);
  std::vector<int64_t> steps(S->n);
  for (int r = 0; r < S->n; ++r) {
    cur[r] = *S->view[r].cur;
    steps[r] = *S->view[r].steps;
    *S->view[r].cur = start;
  }
  const int64_t saved = S->steps;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    for (int k = 0; k < len; ++k) enqueue_slab_step(S, cs);
    if (hipStreamEndCapture(cs, &g) == hipSuccess && g) {
      if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) ge = nullptr;
      hipGraphDestroy(g);
    }
  }
  for (int r = 0; r < S->n; ++r) {
    *S->view[r].cur = cur[r];
    *S->view[r].steps = steps[r];
  }
  S->steps = saved;
  hipStreamDestroy(cs);
  hipGetLastError();
  return ge;
}

int slab_check(imb_slab* S, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return slab_fail(S, e, what);
  return IMB_OK;
}

int slab_sync(imb_slab* S) {
  for (int r = 0; r < S->n; ++r) {
    const int rc = imb_sync(S->rank[r]);
    if (rc) {
      S->err = std::string("slab ") + std::to_string(r) + ": " + imb_last_error(S->rank[r]);
      return rc;
    }
  }
  return IMB_OK;
}

int slab_stage(imb_slab* S, size_t bytes) {
  if (S->stage_bytes >= bytes) return IMB_OK;
  hipStreamSynchronize(S->stream);
  if (S->stage) hipFree(S->stage);
  S->stage = nullptr;
  S->stage_bytes = 0;
  hipError_t e = hipMalloc((void**)&S->stage, bytes);
  if (e != hipSuccess) {
    S->stage = nullptr;
    S->err = "hipMalloc(staging) failed";
    return IMB_ENOMEM;
  }
  S->stage_bytes = bytes;
  return IMB_OK;
}

size_t elem_bytes(int storage) {
  return storage == IMB_STORAGE_F64 ? 8 : (storage == IMB_STORAGE_F32 ? 4 : 2);
}

}  // namespace

extern "C" {

int imb_slab_create(const imb_config* cfg, int32_t nslabs, void* hip_stream, imb_slab** out) {
  if (!out) return IMB_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = validate_config(cfg, &why);
  if (rc) {
    g_slab_create_error = why;
    return rc;
  }
  if (nslabs < 2 || nslabs > MAX_SLABS) {
    g_slab_create_error = "nslabs must be in 2..16";
    return IMB_EINVAL;
  }
  Geometry g;
  sim_geometry(*cfg, &g);
  const int trows = g.tiles_y;  // tile rows of the lattice, shared out between the slabs
  if (trows < nslabs) {
    g_slab_create_error = "more slabs than tile rows";
    return IMB_EINVAL;
  }
  imb_slab* S = new (std::nothrow) imb_slab();
  if (!S) return IMB_ENOMEM;
  S->cfg = *cfg;
  if (!S->cfg.tile_w) S->cfg.tile_w = 64;
  if (!S->cfg.tile_rows) S->cfg.tile_rows = 1;
  S->n = nslabs;
  S->stream = (hipStream_t)hip_stream;
  const bool walls = cfg->flags & IMB_FLAG_WALLS;
  int t0 = 0;
  for (int r = 0; r < nslabs; ++r) {
    const int nt = trows / nslabs + (r < trows % nslabs ? 1 : 0);
    S->y0[r] = t0 * g.th;
    S->rows[r] = std::min(cfg->ny - S->y0[r], nt * g.th);
    t0 += nt;
  }
  for (int r = 0; r < nslabs; ++r) {
    imb_sim* s = nullptr;
    rc = create_window_sim(&S->cfg, S->y0[r], S->rows[r], hip_stream, &s);
    if (rc) {
      g_slab_create_error = create_error();
      imb_slab_destroy(S);
      return rc;
    }
    S->rank.push_back(s);
    S->view.push_back(sim_view(s));
  }
  // A slab face is a wall or a neighbour; the lowest and highest slabs meet each other across
  // the periodic boundary.  Window row j is plane row j + 1.  The ghost row below slab r (plane
  // row 0) takes the populations 2, 5, 6 of the last row of the slab below (its plane row
  // rows_below); the ghost row above (plane row rows_r + 1) takes 4, 7, 8 of the first row of
  // the slab above (its plane row 1).
  std::vector<RowCopy> tab[2];
  const size_t es = elem_bytes(cfg->storage);
  for (int r = 0; r < nslabs; ++r) {
    const bool has_lo = !(walls && r == 0);
    const bool has_hi = !(walls && r == nslabs - 1);
    set_window_ghosts(S->rank[r], has_lo, has_hi);
    const int below = (r + nslabs - 1) % nslabs, above = (r + 1) % nslabs;
    const Geometry& gr = *S->view[r].g;
    for (int k = 0; k < 2; ++k) {
      auto row = [&](int slab, int q, int prow) {
        const Geometry& gs = *S->view[slab].g;
        return (char*)S->view[slab].d->f[k] +
               ((size_t)q * gs.plane + (size_t)prow * gs.pitch) * es;
      };
      static constexpr int up[3] = {2, 5, 6}, down[3] = {4, 7, 8};
      for (int j = 0; j < 3; ++j) {
        if (has_lo) tab[k].push_back({row(below, up[j], S->rows[below]), row(r, up[j], 0)});
        if (has_hi)
          tab[k].push_back({row(above, down[j], 1), row(r, down[j], gr.nyl + 1)});
      }
    }
  }
  const size_t ncopy = tab[0].size();
  const size_t tab_bytes = align_up(std::max(ncopy, (size_t)1) * sizeof(RowCopy), 256);
  const size_t mp = (size_t)std::max(cfg->max_particles, 1);
  const size_t bytes = 2 * tab_bytes + mp * DISK_PARTS * sizeof(double4);
  hipError_t e = hipMalloc((void**)&S->xmem, bytes);
  if (e != hipSuccess) {
    S->xmem = nullptr;
    g_slab_create_error = "hipMalloc(slab exchange) failed";
    imb_slab_destroy(S);
    return IMB_ENOMEM;
  }
  launch_fill_zero(S->xmem, bytes, S->stream);
  S->fsum = (double4*)(S->xmem + 2 * tab_bytes);
  const size_t row_bytes = (size_t)cfg->nx * es;
  for (int k = 0; k < 2; ++k) {
    RowCopy* dtab = (RowCopy*)(S->xmem + k * tab_bytes);
    if (ncopy) {
      e = hipMemcpyAsync(dtab, tab[k].data(), ncopy * sizeof(RowCopy), hipMemcpyHostToDevice,
                         S->stream);
      if (e != hipSuccess) {
        g_slab_create_error = "hipMemcpyAsync(row-copy table) failed";
        imb_slab_destroy(S);
        return IMB_EHIP;
      }
    }
    ExchangeArgs& x = S->xa[k];
    x.copy = dtab;
    x.ncopy = (int)ncopy;
    x.half_words = row_bytes % 4 != 0;
    x.words = (int)(row_bytes / (x.half_words ? 2 : 4));
    x.nslab = nslabs;
    for (int r = 0; r < nslabs; ++r) x.part[r] = S->view[r].d->force;
    x.sum = S->fsum;
  }
  hipStreamSynchronize(S->stream);  // the host tables are released on return
  const int work = std::max(S->xa[0].words, (int)mp);  // per block row
  S->xgrid = std::max(1, std::min((work + 255) / 256, 64));
  rc = imb_slab_init_equilibrium(S, cfg->rho0, 0.0, 0.0);
  if (rc) {
    g_slab_create_error = S->err;
    imb_slab_destroy(S);
    return rc;
  }
  *out = S;
  return IMB_OK;
}

void imb_slab_destroy(imb_slab* S) {
  if (!S) return;
  if (S->stream || !S->rank.empty()) hipStreamSynchronize(S->stream);
  drop_slab_graphs(S);
  for (auto& t : S->timed) {
    hipEventDestroy(t.e0);
    hipEventDestroy(t.e1);
  }
  for (auto e : S->ev_pool) hipEventDestroy(e);
  for (auto* s : S->rank) imb_destroy(s);
  if (S->xmem) hipFree(S->xmem);
  if (S->stage) hipFree(S->stage);
  delete S;
}

int imb_slab_layout(const imb_slab* S, int32_t* y0, int32_t* rows) {
  if (!S || !y0 || !rows) return IMB_EINVAL;
  for (int r = 0; r < S->n; ++r) {
    y0[r] = S->y0[r];
    rows[r] = S->rows[r];
  }
  return IMB_OK;
}

int imb_slab_init_equilibrium(imb_slab* S, double rho, double ux, double uy) {
  if (!S) return IMB_EINVAL;
  if (!(rho > 0.0) || !std::isfinite(ux) || !std::isfinite(uy)) {
    S->err = "invalid equilibrium state";
    return IMB_EINVAL;
  }
  double feq[NQ];
  const double uu = ux * ux + uy * uy;
  for (int i = 0; i < NQ; ++i) {
    const double cu = (double)cx_of(i) * ux + (double)cy_of(i) * uy;
    feq[i] = w_of(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
  drop_slab_graphs(S);
  for (int r = 0; r < S->n; ++r) {
    LatticeArgs a = lattice_args(S->rank[r], nullptr, nullptr);
    launch_unstream(S->cfg.storage, a, nullptr, feq, S->view[r].d->f[*S->view[r].cur],
                    S->stream);
  }
  const int rc = slab_check(S, "init_equilibrium");
  return rc ? rc : slab_sync(S);
}

int imb_slab_set_populations(imb_slab* S, const double* host_f) {
  if (!S || !host_f) return IMB_EINVAL;
  const size_t n = (size_t)NQ * S->cfg.nx * S->cfg.ny;
  int rc = slab_stage(S, n * sizeof(double));
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(S->stage, host_f, n * sizeof(double), hipMemcpyHostToDevice,
                                S->stream);
  if (e != hipSuccess) return slab_fail(S, e, "hipMemcpyAsync");
  for (int r = 0; r < S->n; ++r) {  // each slab's rows and both ghost rows
    LatticeArgs a = lattice_args(S->rank[r], nullptr, nullptr);
    launch_unstream(S->cfg.storage, a, S->stage, nullptr, S->view[r].d->f[*S->view[r].cur],
                    S->stream);
  }
  rc = slab_check(S, "set_populations");
  return rc ? rc : slab_sync(S);
}

static int slab_gather(imb_slab* S, double* fq, double* rho, double* ux, double* uy) {
  for (int r = 0; r < S->n; ++r) {
    LatticeArgs a = lattice_args(S->rank[r], nullptr, nullptr);
    launch_gather(S->cfg.storage, a, S->view[r].d->f[*S->view[r].cur], fq, rho, ux, uy,
                  S->stream);
  }
  return slab_check(S, "gather");
}

int imb_slab_get_populations(imb_slab* S, double* host_f) {
  if (!S || !host_f) return IMB_EINVAL;
  const size_t n = (size_t)NQ * S->cfg.nx * S->cfg.ny;
  int rc = slab_stage(S, n * sizeof(double));
  if (!rc) rc = slab_gather(S, S->stage, nullptr, nullptr, nullptr);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(host_f, S->stage, n * sizeof(double), hipMemcpyDeviceToHost,
                                S->stream);
  if (e != hipSuccess) return slab_fail(S, e, "hipMemcpyAsync");
  return slab_sync(S);
}

int imb_slab_get_fields(imb_slab* S, double* rho, double* ux, double* uy) {
  if (!S) return IMB_EINVAL;
  const size_t n = (size_t)S->cfg.nx * S->cfg.ny;
  int rc = slab_stage(S, 3 * n * sizeof(double));
  if (!rc) rc = slab_gather(S, nullptr, S->stage, S->stage + n, S->stage + 2 * n);
  if (rc) return rc;
  double* outs[3] = {rho, ux, uy};
  for (int k = 0; k < 3; ++k) {
    if (!outs[k]) continue;
    hipError_t e = hipMemcpyAsync(outs[k], S->stage + k * n, n * sizeof(double),
                                  hipMemcpyDeviceToHost, S->stream);
    if (e != hipSuccess) return slab_fail(S, e, "hipMemcpyAsync");
  }
  return slab_sync(S);
}

int imb_slab_set_particles(imb_slab* S, int32_t n, const double* x, const double* y,
                           const double* r, const double* vx, const double* vy, const double* om,
                           const int32_t* mode) {
  if (!S) return IMB_EINVAL;
  hipStreamSynchronize(S->stream);
  drop_slab_graphs(S);
  for (int k = 0; k < S->n; ++k) {  // the same disks on every slab (replicated particle phase)
    const int rc = imb_set_particles(S->rank[k], n, x, y, r, vx, vy, om, mode);
    if (rc) {
      S->err = imb_last_error(S->rank[k]);
      return rc;
    }
  }
  S->np = n;
  S->xa[0].np = S->xa[1].np = n;
  return IMB_OK;
}

int imb_slab_step(imb_slab* S, int32_t nsteps) {
  if (!S || nsteps < 0) return IMB_EINVAL;
  if (S->timing) {
    for (int k = 0; k < nsteps; ++k) enqueue_slab_step(S, S->stream);
    return slab_check(S, "step");
  }
  while (nsteps > 0) {
    const int li = nsteps >= SLAB_GRAPH_LONG ? 1 : (nsteps >= 2 ? 0 : -1);
    if (li < 0) {
      enqueue_slab_step(S, S->stream);
      --nsteps;
      continue;
    }
    const int len = li ? SLAB_GRAPH_LONG : 2;
    const int c = *S->view[0].cur;
    if (!S->graph[li][c]) S->graph[li][c] = capture_slab_steps(S, len, c);
    if (!S->graph[li][c]) {  // capture unavailable: launch directly
      for (int k = 0; k < len; ++k) enqueue_slab_step(S, S->stream);
    } else {
      hipError_t e = hipGraphLaunch(S->graph[li][c], S->stream);
      if (e != hipSuccess) return slab_fail(S, e, "hipGraphLaunch");
      for (int r = 0; r < S->n; ++r) *S->view[r].steps += len;  // even length: parity kept
      S->steps += len;
    }
    nsteps -= len;
  }
  return slab_check(S, "step");
}

int imb_slab_get_forces(imb_slab* S, double* fx, double* fy, double* tz) {
  if (!S) return IMB_EINVAL;
  const int rc = imb_get_forces(S->rank[0], fx, fy, tz);
  if (rc) S->err = imb_last_error(S->rank[0]);
  return rc;
}

int imb_slab_get_partial_forces(imb_slab* S, int32_t slab, double* fx, double* fy, double* tz) {
  if (!S || slab < 0 || slab >= S->n) return IMB_EINVAL;
  std::vector<double4> h((size_t)std::max(S->np, 1) * DISK_PARTS);
  if (S->np > 0) {
    hipError_t e = hipMemcpyAsync(h.data(), S->view[slab].d->force,
                                  (size_t)S->np * DISK_PARTS * sizeof(double4),
                                  hipMemcpyDeviceToHost, S->stream);
    if (e != hipSuccess) return slab_fail(S, e, "hipMemcpyAsync");
  }
  const int rc = slab_sync(S);
  if (rc) return rc;
  for (int p = 0; p < S->np; ++p) {  // the slab's share: its two workgroups' parts added
    const double4 u = h[DISK_PARTS * p], v = h[DISK_PARTS * p + 1];
    if (fx) fx[p] = u.x + v.x;
    if (fy) fy[p] = u.y + v.y;
    if (tz) tz[p] = u.z + v.z;
  }
  return IMB_OK;
}

int imb_slab_get_particles(imb_slab* S, int32_t slab, double* x, double* y, double* vx,
                           double* vy, double* om) {
  if (!S || slab < 0 || slab >= S->n) return IMB_EINVAL;
  const int rc = imb_get_particles(S->rank[slab], x, y, vx, vy, om);
  if (rc) S->err = imb_last_error(S->rank[slab]);
  return rc;
}

int imb_slab_set_kernel_timing(imb_slab* S, int enable) {
  if (!S) return IMB_EINVAL;
  hipStreamSynchronize(S->stream);
  S->timing = enable != 0;
  for (int r = 0; r < S->n; ++r) S->lat_ms[r] = S->par_ms[r] = 0.0;
  S->xch_ms = 0.0;
  S->timed_steps = 0;
  for (auto& t : S->timed) {
    S->ev_pool.push_back(t.e0);
    S->ev_pool.push_back(t.e1);
  }
  S->timed.clear();
  return IMB_OK;
}

int imb_slab_get_kernel_timing(imb_slab* S, double* lattice_ms, double* exchange_ms,
                               double* particle_ms, int64_t* nsteps) {
  if (!S) return IMB_EINVAL;
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return slab_fail(S, e, "hipStreamSynchronize");
  for (auto& t : S->timed) {
    float ms = 0.0f;
    hipEventElapsedTime(&ms, t.e0, t.e1);
    if (t.kind == 0) S->lat_ms[t.slab] += ms;
    else if (t.kind == 1) {
      S->xch_ms += ms;
      S->timed_steps++;
    } else S->par_ms[t.slab] += ms;
    S->ev_pool.push_back(t.e0);
    S->ev_pool.push_back(t.e1);
  }
  S->timed.clear();
  for (int r = 0; r < S->n; ++r) {
    if (lattice_ms) lattice_ms[r] = S->lat_ms[r];
    if (particle_ms) particle_ms[r] = S->par_ms[r];
  }
  if (exchange_ms) *exchange_ms = S->xch_ms;
  if (nsteps) *nsteps = S->timed_steps;
  return IMB_OK;
}

int imb_slab_sync(imb_slab* S) {
  if (!S) return IMB_EINVAL;
  return slab_sync(S);
}

const char* imb_slab_last_error(const imb_slab* S) {
  return S ? S->err.c_str() : g_slab_create_error.c_str();
}

}  // extern "C"

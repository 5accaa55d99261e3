// batch.hip -- batched form: many independent channels (each its own lattice size, disks,
// relaxation time) advanced by ONE persistent kernel per imb_batch_step call, captured in a
// hipGraph and replayed.
//
// Schedule.  The channels are split into two halves A and B of about equal tile counts.  A step
// n is two phases separated by grid-wide barriers:
//     phase 2n    : lattice tiles of A at step n      + particle phases of B for step n - 1
//     phase 2n + 1: lattice tiles of B at step n      + particle phases of A for step n
// (a last phase runs B's particle phase of the last step).  A channel's particle phase (force
// finalisation, DEM, disk tables) thus always runs while the other half streams its lattice, so
// the one-workgroup DEM never idles the grid, and every dependency (tiles of a step -> that
// step's particle phase -> the next step's tiles) crosses at least one barrier.  Inside a phase
// the workgroups pull tickets from an atomic counter: the half's particle phases first (the
// long items), then chunks of DISK_CHUNK (channel, disk) items (a disk's covered cells and
// force), then chunks of TILE_CHUNK (channel, tile) items (the uncovered cells), each in channel
// order; chunking keeps the number of increments of the one counter small.
//
// The persistent grid is sized to the number of co-resident workgroups; every wait is bounded
// (a barrier that does not open within the time limit sets an abort flag that every workgroup
// checks, so the kernel always drains and the host reports the failure).
//
// Each channel is an ordinary simulation handle whose memory is carved from the batch buffer
// with room for any tile shape; the lattice tile and the particle phase are the same device code
// as the single-channel kernels, so a channel in a batch evolves bit for bit like the same
// channel run alone with the same tile shape.
#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

#include "disk_block.h"
#include "particle_phase.h"
#include "runtime.h"

namespace imb {

constexpr int MAX_BATCH = 128;   // channels per batch
// Disks per channel: the persistent kernel runs a channel's particle phase in one of its own
// 256-thread workgroups (one disk per thread), so it takes channels of at most 256 disks; the
// per-step schedule launches the particle phases on their own and takes up to MAX_PARTICLES with
// 512-thread workgroups, as a single simulation does.
constexpr int PERSISTENT_MAX_DISKS = BLOCK;
constexpr int PP_LDS = PERSISTENT_MAX_DISKS * PP_DOUBLES;  // doubles of particle-phase scratch
constexpr int PP_WIDE = MAX_PARTICLES;                     // threads of the wide particle phase
constexpr int PP_LDS_WIDE = PP_WIDE * PP_DOUBLES;
constexpr int SYNC_WORDS = 8;    // [0] arrivals [1] generation [2],[3] item counters [4] abort
constexpr int TILE_CHUNK = 8;    // consecutive tiles taken with one atomic increment
constexpr int DISK_CHUNK = 2;    // consecutive disks taken with one atomic increment

// Arguments of one channel for a step reading buffer k (la[k]: buffer k to buffer k ^ 1 with the
// disk tables of slot k; pa[k]: that step's particle phase, writing the tables of slot k ^ 1).
struct BatchChannel {
  LatticeArgs la[2];
  ParticleArgs pa[2];
};

struct BatchArgs {
  const int* half_ch;    // [2][MAX_BATCH] channels of each half
  const int* half_pref;  // [2][MAX_BATCH + 1] tile prefix sums of each half
  const int* half_dpref; // [2][MAX_BATCH + 1] disk prefix sums of each half
  int half_n0, half_n1, half_t0, half_t1, half_d0, half_d1;
  int nsteps, parity0, nblocks;
  unsigned* sync;
  long long spin_ticks;  // longest barrier wait, wall-clock ticks
};

__device__ inline unsigned ld_agent(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier (generation counter).  The last arriving workgroup clears the arrival count
// and the finished phase's item counter, then opens the next generation.  Returns false when the
// batch was aborted (a wait exceeded the limit here or elsewhere).
__device__ bool grid_barrier(unsigned* sync, int nblocks, int reset_word, long long spin_ticks) {
  __shared__ int s_ok;
  // Every wave waits until its own stores have reached the L2 (a workgroup barrier alone does
  // not wait for global stores); thread 0 then releases them device-wide and arrives.  The
  // agent-scope fence writes back the whole L2 of the compute die, so it is issued once per
  // workgroup rather than once per wave.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    int ok = 1;
    const unsigned gen = ld_agent(&sync[1]);
    const unsigned arrived = atomicAdd(&sync[0], 1u);
    if (arrived == (unsigned)nblocks - 1u) {
      __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sync[reset_word], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      atomicAdd(&sync[1], 1u);
    } else {
      const long long t0 = wall_clock64();
      while (ld_agent(&sync[1]) == gen) {
        if (ld_agent(&sync[4])) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > spin_ticks) {
          atomicOr(&sync[4], 1u);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __threadfence();  // acquire: what other workgroups released is visible to this workgroup
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Channel slot k of half h holding item i of a prefix table: the last k < n with pref[k] <= i
// (channels whose range is empty are skipped).
__device__ inline int find_slot(const int* pref, int n, int i) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pref[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ch: the channel table (read-only during the launch; the channel and item indices are uniform
// over a workgroup, so a channel's arguments are read with scalar loads).
// The persistent kernel calls the particle phase out of line: in-line, its registers would add to
// those of the lattice roles and spill.
__device__ __attribute__((noinline)) void particle_phase_call(const ParticleArgs& a, double* lds) {
  particle_phase<BLOCK>(a, lds);
}

__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3))) void k_batch(
    BatchArgs B, const BatchChannel* __restrict__ ch) {
  __shared__ int s_item, s_abort;
  __shared__ int s_hch[2][MAX_BATCH];
  __shared__ int s_hpref[2][MAX_BATCH + 1];
  __shared__ int s_hdpref[2][MAX_BATCH + 1];
  __shared__ double pp_lds[PP_LDS];
  const int tid = threadIdx.x;
  for (int k = tid; k < MAX_BATCH; k += BLOCK) {
    s_hch[0][k] = B.half_ch[k];
    s_hch[1][k] = B.half_ch[MAX_BATCH + k];
  }
  for (int k = tid; k <= MAX_BATCH; k += BLOCK) {
    s_hpref[0][k] = B.half_pref[k];
    s_hpref[1][k] = B.half_pref[MAX_BATCH + 1 + k];
    s_hdpref[0][k] = B.half_dpref[k];
    s_hdpref[1][k] = B.half_dpref[MAX_BATCH + 1 + k];
  }
  __syncthreads();  // the tables are complete before any wave reads them
  const int hn[2] = {B.half_n0, B.half_n1};
  const int ht[2] = {B.half_t0, B.half_t1};
  const int hd[2] = {B.half_d0, B.half_d1};
  const int nphase = 2 * B.nsteps + 1;
  for (int p = 0; p < nphase; ++p) {
    const int n = p >> 1, h = p & 1;
    const int ph = 1 - h;  // half whose particle phase runs now
    const int npart = (h == 1 || n >= 1) ? hn[ph] : 0;
    const bool lat = p < 2 * B.nsteps;
    const int ndisk = lat ? hd[h] : 0;
    const int nlat = lat ? ht[h] : 0;
    // tickets: one per particle phase, one per DISK_CHUNK disks, one per TILE_CHUNK tiles
    const int ndc = (ndisk + DISK_CHUNK - 1) / DISK_CHUNK;
    const int ntc = (nlat + TILE_CHUNK - 1) / TILE_CHUNK;
    const int par = (B.parity0 + n) & 1;
    unsigned* ctr = &B.sync[2 + (p & 1)];
    for (;;) {
      __syncthreads();
      if (tid == 0) {
        s_item = (int)atomicAdd(ctr, 1u);
        s_abort = (int)ld_agent(&B.sync[4]);
      }
      __syncthreads();
      const int i = __builtin_amdgcn_readfirstlane(s_item);
      if (s_abort || i >= npart + ndc + ntc) break;
      if (i < npart) {  // the particle phase of step n (half B: of step n - 1)
        const int m = h == 1 ? n : n - 1;
        const int ci = __builtin_amdgcn_readfirstlane(s_hch[ph][i]);
        particle_phase_call(ch[ci].pa[(B.parity0 + m) & 1], pp_lds);
        continue;
      }
      const bool is_disk = i < npart + ndc;
      const int chunk = is_disk ? DISK_CHUNK : TILE_CHUNK;
      const int c0 = (is_disk ? i - npart : i - npart - ndc) * chunk;
      const int c1 = min(c0 + chunk, is_disk ? ndisk : nlat);
      for (int t = c0; t < c1; ++t) {  // the chunk's items in order (block-uniform bounds)
        if (t > c0) __syncthreads();   // the previous item's LDS is no longer read
        const int k = find_slot(is_disk ? s_hdpref[h] : s_hpref[h], hn[h], t);
        const int ci = __builtin_amdgcn_readfirstlane(s_hch[h][k]);
        const LatticeArgs la = ch[ci].la[par];
        if (is_disk) {
          disk_cells<StoreF32>(la, t - s_hdpref[h][k]);
        } else {
          fluid_tile<StoreF32>(la, t - s_hpref[h][k]);
        }
      }
    }
    if (p + 1 < nphase && !grid_barrier(B.sync, B.nblocks, 2 + (p & 1), B.spin_ticks)) return;
  }
}

// Per-step schedule: the lattice part of every channel as one ordinary launch (the disk items
// of all channels first, then their tiles; the same device code as k_step), then one
// particle-phase workgroup per channel.  No grid barrier and no device-wide fence: the kernel
// boundaries order the steps.  The tiles of all channels, concatenated in channel order, are
// handed out XCD-aware (each XCD takes a contiguous run of them, so tiles that share rows and
// halo lines share an L2).
// Workgroup b finds its channel and item in one scalar load from a table built on the host
// (a search over the channels' prefix sums took a chain of dependent loads per workgroup).  The
// channel index is uniform over the workgroup and the tables are read-only during the launch,
// so a channel's arguments are read with scalar loads instead of occupying vector registers.
// Held to six wavefronts per SIMD (80 VGPRs) like the single-simulation lattice kernel.
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_batch_lattice(
    const BatchChannel* __restrict__ ch, const unsigned* __restrict__ blk, int ndisk, int ntile,
    int parity) {
  const int b = blockIdx.x;
  const int j = b < ndisk ? b : ndisk + xcd_remap(b - ndisk, ntile);
  const unsigned e = __builtin_amdgcn_readfirstlane(blk[j]);  // (channel << 24) | item
  const LatticeArgs la = ch[e >> 24].la[parity];
  const int item = (int)(e & 0xFFFFFFu);
  if (b < ndisk) disk_cells<StoreF32>(la, item);
  else fluid_tile<StoreF32>(la, item);
}

__global__ __launch_bounds__(BLOCK) void k_batch_particles(const BatchChannel* __restrict__ ch,
                                                           int parity) {
  __shared__ double pp_lds[PP_LDS];
  particle_phase<BLOCK>(ch[blockIdx.x].pa[parity], pp_lds);
}

// The same for batches holding a channel of more than PERSISTENT_MAX_DISKS disks (per-step
// schedule only).
__global__ __launch_bounds__(PP_WIDE) void k_batch_particles_wide(
    const BatchChannel* __restrict__ ch, int parity) {
  __shared__ double pp_lds[PP_LDS_WIDE];
  particle_phase<PP_WIDE>(ch[blockIdx.x].pa[parity], pp_lds);
}

}  // namespace imb

using namespace imb;

struct imb_batch {
  int nch = 0;
  std::vector<imb_sim*> sims;
  std::vector<size_t> offs;
  hipStream_t stream = nullptr;
  char* mem = nullptr;
  size_t mem_bytes = 0;
  bool owns = false;
  BatchChannel* d_ch = nullptr;
  int* d_half = nullptr;
  unsigned* d_blk = nullptr;  // per-step schedule: (channel << 24) | item of every disk item and
                              // tile, all channels' disk items first, then their tiles
  size_t blk_cap = 0;         // entries d_blk holds (the finest tile shape's count)
  unsigned* d_sync = nullptr;
  std::vector<BatchChannel> h_ch;
  std::vector<int> h_half;
  int half_n[2] = {0, 0}, half_t[2] = {0, 0}, half_d[2] = {0, 0};
  int all_d = 0, all_t = 0;    // disk items (dparts per disk) and tiles of all channels
  int schedule = IMB_BATCH_PERSISTENT;
  bool wide = false;          // a channel holds more disks than the persistent kernel takes
  int grid = 0, grid_user = 0, occupancy = 0;
  int tile_w = 32, tile_rows = 2;
  int cur = 0;
  bool dirty = true;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  hipEvent_t ev[2] = {nullptr, nullptr};
  float last_ms = 0.f;
  int64_t steps = 0;
  std::string err;
};

namespace {

thread_local std::string g_batch_error;

imb_config layout_config(const imb_config& c) {
  imb_config l = c;  // the most band-mask rows any tile shape can need
  l.tile_w = 256;
  l.tile_rows = 1;
  return l;
}

int validate_batch(int32_t nsim, const imb_config* cfgs, std::string* why) {
  if (nsim < 1 || nsim > MAX_BATCH || !cfgs) {
    *why = "batch needs 1.." + std::to_string(MAX_BATCH) + " configurations";
    return IMB_EINVAL;
  }
  for (int c = 0; c < nsim; ++c) {
    std::string w;
    if (validate_config(&cfgs[c], &w)) {
      *why = "channel " + std::to_string(c) + ": " + w;
      return IMB_EINVAL;
    }
    if (cfgs[c].storage != IMB_STORAGE_F32) {
      *why = "channel " + std::to_string(c) + ": batched channels use F32 storage";
      return IMB_EUNSUPPORTED;
    }
    imb_config l = layout_config(cfgs[c]);
    if (validate_config(&l, &w)) {
      *why = "channel " + std::to_string(c) + ": " + w;
      return IMB_EINVAL;
    }
  }
  return IMB_OK;
}

// Entries of the per-step schedule's workgroup table: every channel's disk items and its tiles
// under the tile shape with the most tiles.
size_t block_table_entries(int nsim, const imb_config* cfgs) {
  size_t n = 0;
  for (int c = 0; c < nsim; ++c) {
    size_t most = 0;
    for (int tw = 16; tw <= 256; tw *= 2)
      for (int rows = 1; rows <= 4; rows *= 2) {
        imb_config t = cfgs[c];
        t.tile_w = tw;
        t.tile_rows = rows;
        Geometry g;
        sim_geometry(t, &g);
        most = std::max(most, (size_t)g.tiles_x * g.tiles_y);
      }
    n += (size_t)std::max(cfgs[c].max_particles, 1) * DISK_PARTS + most;
  }
  return n;
}

size_t table_bytes(int nsim, const imb_config* cfgs) {
  return align_up(sizeof(BatchChannel) * nsim, 256) +
         align_up(sizeof(int) * 2 * (3 * MAX_BATCH + 2), 256) +
         align_up(sizeof(unsigned) * SYNC_WORDS, 256) +
         align_up(sizeof(unsigned) * block_table_entries(nsim, cfgs), 256);
}

void drop_batch_graphs(imb_batch* b) {
  for (auto& kv : b->graphs)
    if (kv.second) hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// Halves of about equal tile counts (largest channels first, each to the lighter half), the
// per-channel kernel arguments, uploaded to the device.
int refresh(imb_batch* b) {
  if (!b->dirty) return IMB_OK;
  drop_batch_graphs(b);
  b->h_ch.assign(b->nch, BatchChannel{});
  std::vector<int> order(b->nch), tiles(b->nch);
  for (int c = 0; c < b->nch; ++c) {
    imb_sim* s = b->sims[c];
    SimView v = sim_view(s);
    for (int k = 0; k < 2; ++k) {
      ParticleArgs pa = particle_args(s, k ^ 1);
      pa.do_finalize = 1;
      pa.do_dem = 1;
      pa.do_table = 1;
      pa.lds_doubles = b->wide ? PP_LDS_WIDE : PP_LDS;
      b->h_ch[c].la[k] = lattice_args(s, v.d->f[k], v.d->f[k ^ 1]);
      b->h_ch[c].pa[k] = pa;
    }
    tiles[c] = v.g->tiles_x * v.g->tiles_y;
    order[c] = c;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return tiles[a] > tiles[c]; });
  std::vector<int> hc[2];
  long long load[2] = {0, 0};
  for (int c : order) {
    const int h = load[0] <= load[1] ? 0 : 1;
    hc[h].push_back(c);
    load[h] += tiles[c];
  }
  for (int h = 0; h < 2; ++h) std::sort(hc[h].begin(), hc[h].end());
  b->h_half.assign(2 * (3 * MAX_BATCH + 2), 0);
  int* hch = b->h_half.data();
  int* hpref = hch + 2 * MAX_BATCH;
  int* hdpref = hpref + 2 * (MAX_BATCH + 1);
  for (int h = 0; h < 2; ++h) {
    int acc = 0, dacc = 0;
    for (size_t k = 0; k < hc[h].size(); ++k) {
      hch[h * MAX_BATCH + k] = hc[h][k];
      hpref[h * (MAX_BATCH + 1) + k] = acc;
      hdpref[h * (MAX_BATCH + 1) + k] = dacc;
      acc += tiles[hc[h][k]];
      dacc += b->h_ch[hc[h][k]].la[0].np * b->h_ch[hc[h][k]].la[0].dparts;  // disk items
    }
    for (size_t k = hc[h].size(); k <= (size_t)MAX_BATCH; ++k) {
      hpref[h * (MAX_BATCH + 1) + k] = acc;
      hdpref[h * (MAX_BATCH + 1) + k] = dacc;
    }
    b->half_n[h] = (int)hc[h].size();
    b->half_t[h] = acc;
    b->half_d[h] = dacc;
  }
  // all channels in order (per-step schedule): disk items, then tiles
  b->all_d = 0;
  b->all_t = 0;
  for (int c = 0; c < b->nch; ++c) {
    b->all_d += b->h_ch[c].la[0].np * b->h_ch[c].la[0].dparts;
    b->all_t += tiles[c];
  }
  if ((size_t)b->all_d + b->all_t > b->blk_cap) {
    b->err = "batch workgroup table too small for the tile shape";
    return IMB_EINVAL;
  }
  for (int c = 0; c < b->nch; ++c)
    if (tiles[c] >= (1 << 24)) {  // a table entry holds the item in its low 24 bits
      b->err = "channel " + std::to_string(c) + ": more than 2^24 tiles";
      return IMB_EINVAL;
    }
  std::vector<unsigned> blk((size_t)b->all_d + b->all_t);
  for (int c = 0, d = 0, t = b->all_d; c < b->nch; ++c) {
    const int nd = b->h_ch[c].la[0].np * b->h_ch[c].la[0].dparts;
    for (int i = 0; i < nd; ++i) blk[d++] = ((unsigned)c << 24) | (unsigned)i;
    for (int i = 0; i < tiles[c]; ++i) blk[t++] = ((unsigned)c << 24) | (unsigned)i;
  }
  hipError_t e = hipMemcpyAsync(b->d_ch, b->h_ch.data(), sizeof(BatchChannel) * b->nch,
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_half, b->h_half.data(), sizeof(int) * b->h_half.size(),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && !blk.empty())
    e = hipMemcpyAsync(b->d_blk, blk.data(), sizeof(unsigned) * blk.size(),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    b->err = std::string("batch table upload: ") + hipGetErrorString(e);
    return IMB_EHIP;
  }
  b->grid = b->grid_user > 0 ? std::min(b->grid_user, b->occupancy) : b->occupancy;
  b->dirty = false;
  return IMB_OK;
}

BatchArgs batch_args(imb_batch* b, int nsteps, int parity) {
  BatchArgs a{};
  a.half_ch = b->d_half;
  a.half_pref = b->d_half + 2 * MAX_BATCH;
  a.half_dpref = b->d_half + 2 * MAX_BATCH + 2 * (MAX_BATCH + 1);
  a.half_n0 = b->half_n[0];
  a.half_n1 = b->half_n[1];
  a.half_t0 = b->half_t[0];
  a.half_t1 = b->half_t[1];
  a.half_d0 = b->half_d[0];
  a.half_d1 = b->half_d[1];
  a.nsteps = nsteps;
  a.parity0 = parity;
  a.nblocks = b->grid;
  a.sync = b->d_sync;
  int rate_khz = 0;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, 0) != hipSuccess ||
      rate_khz <= 0)
    rate_khz = 100000;
  a.spin_ticks = (long long)rate_khz * 1000ll * 2;  // 2 s
  return a;
}

void enqueue_batch(imb_batch* b, int nsteps, int parity, hipStream_t s) {
  launch_fill_zero(b->d_sync, sizeof(unsigned) * SYNC_WORDS, s);
  if (b->schedule == IMB_BATCH_PER_STEP) {
    for (int n = 0; n < nsteps; ++n) {
      const int par = (parity + n) & 1;
      hipLaunchKernelGGL(k_batch_lattice, dim3(b->all_d + b->all_t), dim3(BLOCK), 0, s, b->d_ch,
                         (const unsigned*)b->d_blk, b->all_d, b->all_t, par);
      if (b->wide)
        hipLaunchKernelGGL(k_batch_particles_wide, dim3(b->nch), dim3(PP_WIDE), 0, s, b->d_ch,
                           par);
      else
        hipLaunchKernelGGL(k_batch_particles, dim3(b->nch), dim3(BLOCK), 0, s, b->d_ch, par);
    }
    return;
  }
  BatchArgs a = batch_args(b, nsteps, parity);
  hipLaunchKernelGGL(k_batch, dim3(b->grid), dim3(BLOCK), 0, s, a,
                     (const BatchChannel*)b->d_ch);
}

hipGraphExec_t capture_batch(imb_batch* b, int nsteps, int parity) {
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    enqueue_batch(b, nsteps, parity, cs);
    if (hipStreamEndCapture(cs, &g) == hipSuccess && g) {
      if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) ge = nullptr;
      hipGraphDestroy(g);
    }
  }
  hipStreamDestroy(cs);
  hipGetLastError();
  return ge;
}

void advance_channels(imb_batch* b, int nsteps) {
  b->cur ^= nsteps & 1;
  b->steps += nsteps;
  for (imb_sim* s : b->sims) {
    SimView v = sim_view(s);
    *v.cur = b->cur;
    *v.steps += nsteps;
  }
}

int check_channel(imb_batch* b, int sim) {
  if (!b) return IMB_EINVAL;
  if (sim < 0 || sim >= b->nch) {
    b->err = "channel index out of range";
    return IMB_EINVAL;
  }
  return IMB_OK;
}

int batch_sync(imb_batch* b) {
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    b->err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
    return IMB_EHIP;
  }
  unsigned abort = 0;
  e = hipMemcpy(&abort, b->d_sync + 4, sizeof(unsigned), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    b->err = std::string("hipMemcpy: ") + hipGetErrorString(e);
    return IMB_EHIP;
  }
  if (abort) {
    b->err = "batch kernel aborted: a grid barrier did not open within its time limit";
    return IMB_EHIP;
  }
  for (int c = 0; c < b->nch; ++c) {
    const int rc = sync_and_check(b->sims[c]);
    if (rc) {
      b->err = "channel " + std::to_string(c) + ": " + imb_last_error(b->sims[c]);
      return rc;
    }
  }
  return IMB_OK;
}

int run_steps(imb_batch* b, int nsteps, bool use_graph) {
  int rc = refresh(b);
  if (rc) return rc;
  if (nsteps == 0) return IMB_OK;
  if (use_graph) {
    hipGraphExec_t& ge = b->graphs[{nsteps, b->cur}];
    if (!ge) ge = capture_batch(b, nsteps, b->cur);
    if (ge) {
      const hipError_t e = hipGraphLaunch(ge, b->stream);
      if (e != hipSuccess) {
        b->err = std::string("hipGraphLaunch: ") + hipGetErrorString(e);
        return IMB_EHIP;
      }
      advance_channels(b, nsteps);
      return IMB_OK;
    }
  }
  enqueue_batch(b, nsteps, b->cur, b->stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    b->err = std::string("batch launch: ") + hipGetErrorString(e);
    return IMB_EHIP;
  }
  advance_channels(b, nsteps);
  return IMB_OK;
}

int set_shape(imb_batch* b, int tile_w, int tile_rows) {
  for (int c = 0; c < b->nch; ++c) {
    const int rc = set_tile_shape(b->sims[c], tile_w, tile_rows);
    if (rc) {
      b->err = "channel " + std::to_string(c) + ": " + imb_last_error(b->sims[c]);
      return rc;
    }
  }
  b->tile_w = tile_w;
  b->tile_rows = tile_rows;
  b->dirty = true;
  return IMB_OK;
}

}  // namespace

extern "C" {

int imb_batch_required_bytes(int32_t nsim, const imb_config* cfgs, size_t* bytes) {
  if (!bytes) return IMB_EINVAL;
  std::string why;
  const int rc = validate_batch(nsim, cfgs, &why);
  if (rc) return rc;
  size_t total = table_bytes(nsim, cfgs);
  for (int c = 0; c < nsim; ++c) total += align_up(layout(layout_config(cfgs[c]), nullptr, nullptr), 256);
  *bytes = total;
  return IMB_OK;
}

int imb_batch_create(int32_t nsim, const imb_config* cfgs, void* hip_stream, void* dev_buf,
                     size_t dev_bytes, imb_batch** out) {
  if (!out) return IMB_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = validate_batch(nsim, cfgs, &why);
  if (rc) {
    g_batch_error = why;
    return rc;
  }
  size_t need = 0;
  imb_batch_required_bytes(nsim, cfgs, &need);
  imb_batch* b = new (std::nothrow) imb_batch();
  if (!b) return IMB_ENOMEM;
  b->nch = nsim;
  b->stream = (hipStream_t)hip_stream;
  for (int c = 0; c < nsim; ++c)
    if (cfgs[c].max_particles > PERSISTENT_MAX_DISKS) b->wide = true;
  if (b->wide) b->schedule = IMB_BATCH_PER_STEP;
  if (dev_buf) {
    if (dev_bytes < need || ((uintptr_t)dev_buf & 255)) {
      g_batch_error = "bound device buffer too small or not 256-byte aligned";
      delete b;
      return IMB_ENOMEM;
    }
    b->mem = (char*)dev_buf;
  } else {
    if (hipMalloc((void**)&b->mem, need) != hipSuccess) {
      hipGetLastError();
      g_batch_error = "hipMalloc of the batch buffer failed";
      delete b;
      return IMB_ENOMEM;
    }
    b->owns = true;
  }
  b->mem_bytes = need;
  size_t off = 0;
  b->d_ch = (BatchChannel*)(b->mem + off);
  off += align_up(sizeof(BatchChannel) * nsim, 256);
  b->d_half = (int*)(b->mem + off);
  off += align_up(sizeof(int) * 2 * (3 * MAX_BATCH + 2), 256);
  b->d_sync = (unsigned*)(b->mem + off);
  off += align_up(sizeof(unsigned) * SYNC_WORDS, 256);
  b->d_blk = (unsigned*)(b->mem + off);
  b->blk_cap = block_table_entries(nsim, cfgs);
  off += align_up(sizeof(unsigned) * b->blk_cap, 256);
  launch_fill_zero(b->mem, off, b->stream);
  b->tile_w = cfgs[0].tile_w ? cfgs[0].tile_w : 64;
  b->tile_rows = cfgs[0].tile_rows ? cfgs[0].tile_rows : 1;
  for (int c = 0; c < nsim && !rc; ++c) {
    imb_config cc = cfgs[c];
    cc.tile_w = b->tile_w;
    cc.tile_rows = b->tile_rows;
    const imb_config lc = layout_config(cfgs[c]);
    const size_t sz = align_up(layout(lc, nullptr, nullptr), 256);
    imb_sim* s = nullptr;
    rc = create_sim(&cc, &lc, hip_stream, b->mem + off, sz, &s);
    if (rc) {
      g_batch_error = "channel " + std::to_string(c) + ": " + imb_last_error(nullptr);
      break;
    }
    b->sims.push_back(s);
    b->offs.push_back(off);
    off += sz;
  }
  if (!rc) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, BLOCK, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess ||
        per_cu < 1 || cus < 1) {
      hipGetLastError();
      g_batch_error = "cannot size the persistent grid";
      rc = IMB_EHIP;
    } else {
      b->occupancy = per_cu * cus;
    }
  }
  if (!rc) {
    hipEventCreate(&b->ev[0]);
    hipEventCreate(&b->ev[1]);
    rc = refresh(b);
  }
  if (rc) {
    imb_batch_destroy(b);
    return rc;
  }
  *out = b;
  return IMB_OK;
}

void imb_batch_destroy(imb_batch* b) {
  if (!b) return;
  hipStreamSynchronize(b->stream);
  drop_batch_graphs(b);
  for (imb_sim* s : b->sims) imb_destroy(s);
  for (hipEvent_t e : b->ev)
    if (e) hipEventDestroy(e);
  if (b->owns && b->mem) hipFree(b->mem);
  delete b;
}

int imb_batch_set_particles(imb_batch* b, int32_t sim, int32_t n, const double* x,
                            const double* y, const double* r, const double* vx, const double* vy,
                            const double* omega, const int32_t* mode) {
  int rc = check_channel(b, sim);
  if (rc) return rc;
  rc = imb_set_particles(b->sims[sim], n, x, y, r, vx, vy, omega, mode);
  if (rc) b->err = imb_last_error(b->sims[sim]);
  b->dirty = true;
  return rc;
}

int imb_batch_step(imb_batch* b, int32_t nsteps) {
  if (!b || nsteps < 0) return IMB_EINVAL;
  return run_steps(b, nsteps, true);
}

int imb_batch_get_forces(imb_batch* b, int32_t sim, double* fx, double* fy, double* tz) {
  int rc = check_channel(b, sim);
  if (!rc) rc = imb_get_forces(b->sims[sim], fx, fy, tz);
  return rc;
}

int imb_batch_get_particles(imb_batch* b, int32_t sim, double* x, double* y, double* vx,
                            double* vy, double* omega) {
  int rc = check_channel(b, sim);
  if (!rc) rc = imb_get_particles(b->sims[sim], x, y, vx, vy, omega);
  return rc;
}

int imb_batch_get_fields(imb_batch* b, int32_t sim, double* rho, double* ux, double* uy) {
  int rc = check_channel(b, sim);
  if (!rc) rc = imb_get_fields(b->sims[sim], rho, ux, uy);
  return rc;
}

int imb_batch_get_populations(imb_batch* b, int32_t sim, double* host_f) {
  int rc = check_channel(b, sim);
  if (!rc) rc = imb_get_populations(b->sims[sim], host_f);
  return rc;
}

int imb_batch_sync(imb_batch* b) {
  if (!b) return IMB_EINVAL;
  return batch_sync(b);
}

int imb_batch_set_launch(imb_batch* b, int32_t grid, int32_t tile_w, int32_t tile_rows) {
  if (!b || grid < 0) return IMB_EINVAL;
  hipStreamSynchronize(b->stream);
  if (tile_w || tile_rows) {
    const int rc = set_shape(b, tile_w ? tile_w : b->tile_w, tile_rows ? tile_rows : b->tile_rows);
    if (rc) return rc;
  }
  b->grid_user = grid;
  b->dirty = true;
  return refresh(b);
}

int imb_batch_get_launch(imb_batch* b, int32_t* grid, int32_t* tile_w, int32_t* tile_rows,
                         int32_t* max_grid) {
  if (!b) return IMB_EINVAL;
  const int rc = refresh(b);
  if (rc) return rc;
  if (grid) *grid = b->grid;
  if (tile_w) *tile_w = b->tile_w;
  if (tile_rows) *tile_rows = b->tile_rows;
  if (max_grid) *max_grid = b->occupancy;
  return IMB_OK;
}

int imb_batch_set_schedule(imb_batch* b, int32_t schedule) {
  if (!b || (schedule != IMB_BATCH_PERSISTENT && schedule != IMB_BATCH_PER_STEP))
    return IMB_EINVAL;
  if (schedule == IMB_BATCH_PERSISTENT && b->wide) {
    b->err = "the persistent schedule takes at most 256 disks per channel";
    return IMB_EUNSUPPORTED;
  }
  hipStreamSynchronize(b->stream);
  if (schedule != b->schedule) drop_batch_graphs(b);
  b->schedule = schedule;
  return IMB_OK;
}

int imb_batch_get_schedule(imb_batch* b, int32_t* schedule) {
  if (!b || !schedule) return IMB_EINVAL;
  *schedule = b->schedule;
  return IMB_OK;
}

int imb_batch_autotune(imb_batch* b, int32_t trial_steps, double* trial_ms, int32_t max_trials) {
  if (!b || trial_steps < 1) return IMB_EINVAL;
  int rc = batch_sync(b);
  if (rc) return rc;
  // the channels' memory is saved and restored around every trial, so tuning leaves the
  // simulation where it was
  const size_t base = b->offs.front();
  const size_t bytes = b->mem_bytes - base;
  void* save = nullptr;
  if (hipMalloc(&save, bytes) != hipSuccess) {
    hipGetLastError();
    b->err = "autotune: cannot allocate the state snapshot";
    return IMB_ENOMEM;
  }
  launch_copy(save, b->mem + base, bytes, b->stream);
  const int cur0 = b->cur;
  const int64_t steps0 = b->steps;
  std::vector<int64_t> sim_steps0;
  for (imb_sim* s : b->sims) sim_steps0.push_back(*sim_view(s).steps);
  auto restore = [&]() {
    launch_copy(b->mem + base, save, bytes, b->stream);
    b->cur = cur0;
    b->steps = steps0;
    for (int c = 0; c < b->nch; ++c) {
      SimView v = sim_view(b->sims[c]);
      *v.cur = cur0;
      *v.steps = sim_steps0[c];
    }
  };
  static const int shapes[][2] = {{32, 1}, {32, 2}, {32, 4}, {64, 1}, {64, 2}, {64, 4},
                                  {128, 1}, {128, 2}, {16, 4}};
  const int nshapes = (int)(sizeof shapes / sizeof shapes[0]);
  double best = 1e300;
  int bw = b->tile_w, br = b->tile_rows, bg = b->grid_user, bs = b->schedule;
  int done = 0;
  int cu_count = 0;
  hipDeviceGetAttribute(&cu_count, hipDeviceAttributeMultiprocessorCount, 0);
  cu_count = std::max(cu_count, 1);
  for (int k = 0; k < nshapes && rc == IMB_OK; ++k) {
    for (int gsel = 0; gsel < 3 && rc == IMB_OK; ++gsel) {
      if (max_trials > 0 && done >= max_trials) break;
      // per-step schedule; persistent with every co-resident workgroup, or with one workgroup
      // fewer per compute unit
      const int sched = gsel == 0 ? IMB_BATCH_PER_STEP : IMB_BATCH_PERSISTENT;
      const int g = gsel == 2 ? b->occupancy - cu_count : 0;
      if (gsel == 2 && g < cu_count) continue;
      if (sched == IMB_BATCH_PERSISTENT && b->wide) continue;
      // the disk tables were restored with the state: rebuild them for this trial's shape
      if (set_shape(b, shapes[k][0], shapes[k][1]) != IMB_OK) {  // shape not valid here
        restore();
        continue;
      }
      b->grid_user = g;
      b->schedule = sched;
      b->dirty = true;
      rc = run_steps(b, 2, false);  // warm-up
      if (rc) break;
      hipEventRecord(b->ev[0], b->stream);
      rc = run_steps(b, trial_steps, false);
      hipEventRecord(b->ev[1], b->stream);
      if (!rc) rc = batch_sync(b);
      float ms = 0.f;
      hipEventElapsedTime(&ms, b->ev[0], b->ev[1]);
      if (!rc && ms < best) {
        best = ms;
        bw = shapes[k][0];
        br = shapes[k][1];
        bg = g;
        bs = sched;
      }
      restore();
      ++done;
    }
  }
  if (!rc) rc = set_shape(b, bw, br);
  b->grid_user = bg;
  b->schedule = bs;
  b->dirty = true;
  hipStreamSynchronize(b->stream);
  hipFree(save);
  if (!rc) rc = refresh(b);
  if (!rc && trial_ms) *trial_ms = best / trial_steps;
  return rc;
}

int imb_batch_get_timing(imb_batch* b, int32_t nsteps, double* ms) {
  // times nsteps steps (one graph replay) with events; the batch advances by nsteps
  if (!b || nsteps < 1 || !ms) return IMB_EINVAL;
  int rc = batch_sync(b);
  if (rc) return rc;
  rc = refresh(b);
  if (rc) return rc;
  hipEventRecord(b->ev[0], b->stream);
  rc = run_steps(b, nsteps, true);
  hipEventRecord(b->ev[1], b->stream);
  if (!rc) rc = batch_sync(b);
  float t = 0.f;
  hipEventElapsedTime(&t, b->ev[0], b->ev[1]);
  *ms = t;
  return rc;
}

const char* imb_batch_last_error(const imb_batch* b) {
  return b ? b->err.c_str() : g_batch_error.c_str();
}

}  // extern "C"

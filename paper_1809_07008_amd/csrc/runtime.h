// runtime.h -- internal host-side structures shared by runtime.hip, adjoint.hip and batch.hip.
#pragma once

#include <string>

#include "step.h"

namespace imb {

struct Geometry {
  int tw, tw_log, th, rows;  // tile: tw x th cells (th already includes rows)
  int tiles_x, tiles_y;      // tiles of the stored window
  int pitch;
  long long plane;
  // the updated window: rows [y0, y0 + nyl) of the lattice, starting at lattice tile row ty_off
  // of tiles_yg, lattice row y in plane row y - yoff (the whole lattice: 0, ny, 0, 0, tiles_y;
  // a slab's planes hold nyl + 2 rows, a ghost row on each side: yoff = y0 - 1)
  int y0, nyl, yoff, ty_off, tiles_yg;
};

struct DeviceLayout {
  void* f[2];
  ParticleState ps;
  // disk tables, double-buffered: the lattice step whose source populations are f[k] reads
  // tab[k] and band_mask[k]; the particle phase after it writes the other copy, so it can run
  // while the tiles of the same step still read theirs
  ParticleTable tab[2];
  unsigned long long* band_mask[2];  // [MASK_WORDS][tiles_y]
  int* err;
  double* J;
  double* w;  // objective weights wfx, wfy, wtz (3 x capacity)
  unsigned* seed;  // [2] stochastic-rounding step counters
  double4* force;  // [capacity][DISK_PARTS] per-disk force and torque shares of the lattice step
};

struct AdjointState;

// Pointers into an imb_sim for the other translation units.
struct SimView {
  imb_config* cfg;
  Geometry* g;
  DeviceLayout* d;
  hipStream_t stream;
  int* cur;
  int* np;
  int64_t* steps;
  std::string* err;
  AdjointState** adj;
  bool* timing;
  hipStream_t side;
};

size_t align_up(size_t v, size_t a);
// Geometry of the window of `rows` rows from y0 (rows = 0: the whole lattice); y0 must be a
// multiple of the tile height.
void sim_geometry(const imb_config& c, Geometry* g, int y0 = 0, int rows = 0);
size_t layout(const imb_config& c, char* base, DeviceLayout* L, int y0 = 0, int rows = 0);
int validate_config(const imb_config* c, std::string* why);
int hip_fail(std::string* err, hipError_t e, const char* what);
int map_device_error(int bits);
std::string describe_device_error(int bits);

SimView sim_view(imb_sim* s);
LatticeArgs lattice_args(imb_sim* s, const void* src, void* dst);
// Particle-phase arguments writing the disk tables of slot out_slot.
ParticleArgs particle_args(imb_sim* s, int out_slot);
void enqueue_step(imb_sim* s, const double* wfx, const double* wfy, const double* wtz, double* J);
int sync_and_check(imb_sim* s);
int reset_device_error(imb_sim* s);
void free_adjoint(imb_sim* s);
// Forgets a forward pass waiting for its reverse sweep (the disks or the state were replaced).
void disarm_adjoint(imb_sim* s);
void drop_graphs(imb_sim* s);

// Simulation whose memory is carved for `layout_cfg` (same lattice and particle capacity as
// cfg; its tile shape only sets how many tile rows the band masks can hold), so that the tile
// shape can later change in place (set_tile_shape).
int create_sim(const imb_config* cfg, const imb_config* layout_cfg, void* hip_stream,
               void* dev_buf, size_t dev_bytes, imb_sim** out, int win_y0 = 0,
               int win_rows = 0);
// A simulation of the window [y0, y0 + rows) of cfg's lattice (one slab of a lattice split in
// y): its planes hold a ghost row on each side, which its step reads where set_window_ghosts
// says that a neighbouring slab (not a wall) lies there.
int create_window_sim(const imb_config* cfg, int y0, int rows, void* hip_stream, imb_sim** out);
void set_window_ghosts(imb_sim* s, int below, int above);
const char* create_error();
// Changes the tile shape (geometry only; the band capacity must cover the new tile rows) and
// rebuilds the disk tables for it.  Asynchronous.
int set_tile_shape(imb_sim* s, int tile_w, int tile_rows);
int tile_rows_capacity(const imb_sim* s);

}  // namespace imb


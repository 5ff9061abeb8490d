// Internal data structures shared by the host orchestration and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hh {

constexpr int kMaxPhase = 16;

// Solver status values kept per system on the device.
enum : int {
  kRunning = 0,
  kConverged = 1,
  kNoConv = -20,
  kStagnated = -21,
  kBreakdown = -22,
  kNonFinite = -23,
  kSingularStatus = -30,
};

// One image being homogenized in a group of same-shape images.
struct ItemDesc {
  long long lab_off;  // byte offset of the item's labels in the label pack (iso)
  long long cf_off;   // element offset of its 21-component stiffness field (aniso), -1 if iso
  int region[6];      // x0, y0, z0, x1, y1, z1 (half open): the averaging region
  int nphase;
  int pad_;
  double inv_region;  // 1 / |region|
  double lam[kMaxPhase];
  double mu[kMaxPhase];
};

// One linear system = (item, load case).
struct SysDesc {
  int item;
  int load;
};

// Per-system solver state (FP64 scalars).
struct SysState {
  double rr;       // (r, r)
  double bb;       // (b, b)
  double alpha;    // current step length
  double beta;     // current direction update factor
  double best_rr;  // smallest (r, r) seen (stagnation guard)
  double ce2;      // (C:E, C:E), scale of the right-hand side
  double sig[6];   // running < sigma >_R (tensor components 11 22 33 23 13 12)
  double eps[6];   // running < eps >_R
  double sig_best[6];  // averages at the smallest residual seen
  double eps_best[6];
  int iter;
  int status;
  int stall;
  int pad_;
};

// Everything a pass kernel needs about its group of systems.
// Row pitch of the half spectrum: hx rounded up to a multiple of 8, so that
// every row, and every tile of 8 columns, starts on a 128-byte line.
__host__ __device__ constexpr int spectrum_pitch(int hx) { return (hx + 7) / 8 * 8; }

struct GroupArgs {
  int nx, ny, nz, hx;      // grid and half-spectrum length along x
  int hxp;                 // row pitch of the spectrum (spectrum_pitch(hx))
  int nsys;                // systems in this launch
  int nyq_zero;            // 1: operator zero at frequencies with a Nyquist component
  int max_iter;
  int scheme;              // 0 CG, 1 basic fixed point
  int aniso;               // 1: per-voxel 21-component stiffness
  int stall_limit;
  double tol2;             // tol^2
  double zero_rhs2;        // (b,b) below this * (C:E,C:E) counts as zero
  double ref_lam, ref_mu;  // reference medium of the basic scheme
  double loads[6][6];      // loads[a][c]: tensor component c of macroscopic strain a
  const SysDesc* sys;
  const ItemDesc* items;
  const unsigned char* labels;
  const void* cfield;      // T[21] per voxel (aniso)
  void* tmp;               // 6-component half spectrum per system
  void* ar;                // residual, 3-vector form, per system
  void* ap;                // search direction, 3-vector form, per system
  long long tmp_stride;    // complex elements per system
  long long a_stride;      // complex elements per system
  SysState* state;
  double* part_x;          // [nsys][ny * nz rows][kPartX]: row sums of the x pass
  double* part_z;          // [nsys][ny * hx columns]: column sums of the z pass
  double* chunk_x;         // [nsys][nchunk_x][kPartX]: sums of kFinChunk consecutive rows
  double* chunk_z;         // [nsys][nchunk_z]
  int nrow_x, ncol_z;      // ny * nz and ny * hx
  int nchunk_x, nchunk_z;  // ceil(nrow_x / kFinChunk), ceil(ncol_z / kFinChunk)
};

constexpr int kPartX = 13;  // (p, C:p), then region sums of p and of sigma

// Every FP64 reduction of the solve follows a fixed tree defined on the
// grid, not on the tile a workgroup happens to hold, so that all tile
// variants give the same bits:
//  - a line of the x pass (one spectrum row and component pair) is summed
//    in kLineGroups groups, group g taking the line positions g,
//    g + kLineGroups, ... in increasing order, and the groups are added in a
//    fixed butterfly; a column of the z pass likewise in kColGroups groups
//    (one wave), added by a butterfly within each row of 16 lanes and then
//    the four row sums in a fixed order;
//  - the per-row (x) and per-column (z) sums are stored, summed in chunks of
//    kFinChunk consecutive ones by one block each (fixed thread strides and
//    tree), and the chunk sums of a system by one block in a fixed order.
constexpr int kLineGroups = 16;
constexpr int kColGroups = 64;
constexpr int kFinChunk = 4096;

}  // namespace hh

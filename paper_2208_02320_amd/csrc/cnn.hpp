// Internal interface of the CNN surrogate used by the two-level scheme.
#pragma once

#include <hip/hip_runtime.h>

#include "ctx.hpp"

// Predicted stiffness (21 components, denormalized, FP64, device) of `batch`
// items; item i is the n^3 box at offset (o, o, o) of the box^3 labels at
// labels + i * box^3 (device).  counts: label counts of those windows
// ([batch][8], device), or null to count them here.  Every launch goes on st
// (the network's buffers are its own: two networks may run on two streams).
void hh_net_predict_device(hh_ctx* ctx, hh_net* net, const unsigned char* labels, int batch, int box, int o,
                           double* c21, const int* counts, hipStream_t st);
// Whether the network can read its input windows straight from an image of
// nx x ny x nz labels (device), item i being the n^3 block i in C order
// (x fastest): at most four phases, n = 32 or 64, rows on even addresses.
bool hh_net_image_input(const hh_net* net, const unsigned char* img, int nx, int ny);
// As hh_net_predict_device for the nitems blocks of such an image; with
// counts given, st waits for counts_ready (when not null) before the first
// head reads them.
void hh_net_predict_image(hh_ctx* ctx, hh_net* net, const unsigned char* img, int nx, int ny, int nitems,
                          double* c21, const int* counts, hipStream_t st, hipEvent_t counts_ready);
// counts[i][c] = voxels with label c (< 8) in the n^3 window at offset
// (o, o, o) of box i (box^3 labels, device).
void hh_launch_counts(const unsigned char* labels, int nitems, int box, int o, int n, int* counts, hipStream_t st);
// The same for the n^3 blocks of an nx x ny x nz image (item i: block i in C order).
void hh_launch_counts_image(const unsigned char* img, int nx, int ny, int n, int nitems, int* counts,
                            hipStream_t st);
// Phase fractions counts / n^3 -> Voigt and Reuss stiffness (21 components
// each, device).  Cp21/Sp21: per phase stiffness and compliance (21
// components, device).
void hh_launch_bounds(const int* counts, int nitems, int n, int nphase, const double* Cp21, const double* Sp21,
                      double* cv21, double* cr21, hipStream_t st);
// Input-space tests of the gate for one network: label counts of its input
// windows ([nitems][8], device; null switches the tests off), 1 / window
// voxels, the fraction features' mean and scale, the limit z_max, and the
// windows' interface counts (device, may be null) with 1 / pairs per window
// and the training mean and inverse standard deviation of the density.
struct FracGate {
  const int* counts = nullptr;
  double inv_nv = 0.0;
  double mu[8] = {}, sc[8] = {};
  double zmax = 0.0;
  const unsigned* iface = nullptr;
  double inv_pairs = 0.0, imu = 0.0, isc = 0.0;
};
FracGate hh_net_fraction_gate(const hh_net* net, const int* counts, const unsigned* iface);
// Whether the network has interface-density statistics (the gate then needs
// the windows' interface counts).
bool hh_net_has_interface_stats(const hh_net* net);
// counts[i] = face-adjacent voxel pairs with different labels inside the n^3
// window at offset (o, o, o) of box i (box^3 labels, device); zeroes first.
void hh_launch_interfaces(const unsigned char* labels, int nitems, int box, int o, int n, unsigned* counts,
                          hipStream_t st);
// The same for the n^3 blocks of an image; with label_counts ([nitems][8],
// device, or null) the same pass also gives hh_launch_counts_image's counts.
void hh_launch_interfaces_image(const unsigned char* img, int nx, int ny, int n, int nitems, unsigned* counts,
                                hipStream_t st, int* label_counts);
void hh_launch_gate(const double* c21a, const double* c21b, const double* cv21, const double* cr21, int nitems,
                    double spread_tol, double bound_tol, const FracGate& ga, const FracGate& gb, int* flag,
                    hipStream_t st);
int hh_net_input_size(const hh_net* net);

// Host side of the CNN surrogate: parameters, training step, inference, gate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "cnn.hpp"
#include "cnn_kernels.hpp"

using namespace hh::cnn;

namespace {

constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {8, 32, 32, 64};
constexpr int kCout[kLayers] = {32, 32, 64, 64};
constexpr int kFeat = 72, kConvFeat = 64, kFrac = 8, kOut = 21;

struct Buf {
  void* p = nullptr;
  size_t n = 0;
};

}  // namespace

struct hh_net {
  int device = 0;
  int nphase = 0;
  int n = 0;  // input edge
  long long woff[kLayers], boff[kLayers], fcw_off, fcb_off, nparam;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  __bf16* W[kLayers] = {};
  __bf16* Wt[kLayers] = {};
  __bf16* W4 = nullptr;  // first layer by tap pairs (networks of at most four phases)
  __bf16* WR = nullptr;  // first layer by rows of taps (the same networks, even-aligned label rows)
  double mean[kOut], scale[kOut];
  double *d_mean = nullptr, *d_scale = nullptr;
  double fmu[kFrac], fsc[kFrac];  // standardization of the phase-fraction features
  double fzmax = 5.0;              // the gate's limit on |feature| (0: no test)
  double imu = 0.0, isc = 0.0;     // interface density of the training windows (isc 0: no test)
  float *d_fmu = nullptr, *d_fsc = nullptr;
  long long step = 0;
  int cap = 0;  // batch capacity of the activation buffers
  LabelWindow lw{};  // input of the last forward pass (read again by the first layer's weight gradient)
  int* cnt = nullptr;  // label counts per item [cap][8]
  const int* cnt_in = nullptr;  // the counts the head reads (cnt or the caller's)
  __bf16* a[kLayers] = {};
  float* ga[kLayers] = {};  // gradient w.r.t. output of layer l
  float *out = nullptr, *tgt = nullptr, *hw = nullptr, *loss = nullptr;
  float* part = nullptr;
  size_t part_n = 0;
  float* pbias = nullptr;
};

namespace {

int edge(const hh_net* net, int l) { return net->n >> l; }  // input edge of layer l

void free_acts(hh_net* net) {
  (void)hipFree(net->cnt);
  net->cnt = nullptr;
  for (int l = 0; l < kLayers; ++l) {
    (void)hipFree(net->a[l]);
    (void)hipFree(net->ga[l]);
    net->a[l] = nullptr;
    net->ga[l] = nullptr;
  }
  (void)hipFree(net->out);
  (void)hipFree(net->tgt);
  (void)hipFree(net->hw);
  (void)hipFree(net->loss);
  (void)hipFree(net->part);
  (void)hipFree(net->pbias);
  net->out = net->tgt = net->hw = net->loss = net->part = net->pbias = nullptr;
  net->cap = 0;
}

template <class T>
T* dalloc(hh_ctx* ctx, size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(count * sizeof(T), 256)) != hipSuccess) {
    (void)hipGetLastError();
    fail(ctx, HH_ENOMEM, "surrogate: device allocation failed");
  }
  return static_cast<T*>(p);
}

// Voxels per weight-gradient chunk: at most kMaxChunks chunks for any total
// (chunk >= total / kMaxChunks), each a multiple of the 32-voxel MFMA step.
// The first layer's kernel takes all taps per block and so runs more,
// smaller chunks (its partials are 16 times smaller than the last layer's).
constexpr int kMaxChunks = 128, kMaxChunksLab = 1024;

int wgrad_chunk(long long total, int max_chunks) {
  long long c = (total + max_chunks - 1) / max_chunks;
  c = (c + 31) / 32 * 32;
  return int(std::max<long long>(c, 32));
}

void ensure_acts(hh_ctx* ctx, hh_net* net, int batch) {
  if (batch <= net->cap) return;
  // the old buffers may still be read by work queued on any stream
  HIPCHK(hipDeviceSynchronize());
  free_acts(net);
  net->cnt = dalloc<int>(ctx, size_t(batch) * kFrac);
  size_t pmax = 0, bmax = 0;
  for (int l = 0; l < kLayers; ++l) {
    const long long Do = edge(net, l) / 2, nv = Do * Do * Do;
    net->a[l] = dalloc<__bf16>(ctx, size_t(batch) * nv * kCout[l]);
    net->ga[l] = dalloc<float>(ctx, size_t(batch) * nv * kCout[l]);
    // any batch up to the capacity needs at most kMaxChunks partials
    const size_t nc = l == 0 ? kMaxChunksLab : kMaxChunks;
    pmax = std::max<size_t>(pmax, nc * 27 * kCout[l] * kCin[l]);
    bmax = std::max<size_t>(bmax, nc * kCout[l]);
  }
  net->out = dalloc<float>(ctx, size_t(batch) * kOut);
  net->tgt = dalloc<float>(ctx, size_t(batch) * kOut);
  net->hw = dalloc<float>(ctx, size_t(batch) * (kOut * kFeat + kOut));
  net->loss = dalloc<float>(ctx, size_t(batch));
  pmax = std::max<size_t>(pmax, size_t(batch) * (kOut * kFeat + kOut));
  net->part = dalloc<float>(ctx, pmax);
  net->part_n = pmax;
  net->pbias = dalloc<float>(ctx, bmax);
  net->cap = batch;
}

void cast_all(hh_ctx* ctx, hh_net* net) {
  for (int l = 0; l < kLayers; ++l)
    k_cast_weights<<<256, 256, 0, ctx->stream>>>(net->p + net->woff[l], kCin[l], kCout[l], net->W[l], net->Wt[l]);
  k_cast_pairs4<<<16, 256, 0, ctx->stream>>>(net->p + net->woff[0], kCout[0], net->W4);
  k_cast_rows4<<<20, 256, 0, ctx->stream>>>(net->p + net->woff[0], net->p + net->boff[0], kCout[0], net->WR);
  HIPCHK(hipGetLastError());
}

template <int CI, int CO, bool LAB, int RB>
void conv_fwd(hh_ctx* ctx, const __bf16* X, const LabelWindow& lw, const __bf16* W, const float* b, __bf16* Y, int D,
              int batch, hipStream_t st) {
  const int Do = D / 2, nvo = Do * Do * Do;
  const dim3 grid(unsigned((nvo + 64 * RB - 1) / (64 * RB)), unsigned(batch));
  if constexpr (CI == 32 && !LAB) {
    // output rows that tile the 16 lanes of a row block: the x-shift path
    if constexpr (RB == 4) {
      // rows of 16: a wave's row blocks are consecutive rows of one slice;
      // workgroups of 8 waves share the layer's weights through LDS
      if (Do == 16) {
        const dim3 g2(unsigned((nvo + 128 * RB - 1) / (128 * RB)), unsigned(batch));  // 8 waves of 16 RB voxels
        k_conv_fwd<CI, CO, LAB, RB, true, true, 8><<<g2, 512, 0, st>>>(X, lw, W, b, Y, D, make_grid3(Do));
        return;
      }
    }
    if (Do <= 16 && 16 % Do == 0) {
      if constexpr (CO == 64) {
        // 64 output channels (110 KB of weights): workgroups of 16 waves
        // share them through LDS, where an item's output fills such a group
        if (nvo >= 16 * 16 * RB) {
          const dim3 g3(unsigned((nvo + 256 * RB - 1) / (256 * RB)), unsigned(batch));
          k_conv_fwd<CI, CO, LAB, RB, true, false, 16><<<g3, 1024, 0, st>>>(X, lw, W, b, Y, D, make_grid3(Do));
          return;
        }
      }
      k_conv_fwd<CI, CO, LAB, RB, true><<<grid, 256, 0, st>>>(X, lw, W, b, Y, D, make_grid3(Do));
      return;
    }
  }
  k_conv_fwd<CI, CO, LAB, RB><<<grid, 256, 0, st>>>(X, lw, W, b, Y, D, make_grid3(Do));
}

template <int CI, int CO>
void conv_fwd_splitk(hh_ctx* ctx, const __bf16* X, const __bf16* W, const float* b, __bf16* Y, int D, int batch,
                     hipStream_t st) {
  const int Do = D / 2, nvo = Do * Do * Do;
  // four row blocks per workgroup (an item's 4^3 outputs): a quarter of the
  // weight traffic of one
  constexpr int RB = 4;
  if (nvo >= 16 * RB)
    k_conv_fwd_splitk<CI, CO, RB><<<dim3(unsigned((nvo + 16 * RB - 1) / (16 * RB)), unsigned(batch)), 256, 0, st>>>(
        X, W, b, Y, D, make_grid3(Do));
  else
    k_conv_fwd_splitk<CI, CO><<<dim3(unsigned((nvo + 15) / 16), unsigned(batch)), 256, 0, st>>>(
        X, W, b, Y, D, make_grid3(Do));
}

// Whether every window row of lw starts on a w-aligned address.
bool rows_aligned(const LabelWindow& lw, int n, int w) {
  const long long step = lw.mx > 0 ? n : lw.stride;  // from one item's window to the next, along x
  return lw.row % w == 0 && lw.plane % w == 0 && step % w == 0 &&
         reinterpret_cast<uintptr_t>(window_base(lw, 0)) % unsigned(w) == 0;
}

// Whether the first layer reads windows of lw from LDS-staged footprints
// (k_conv_fwd_rows4s): at most four phases, output edges 16 and 32, rows on
// even addresses.  Image windows need it.
bool staged_first_layer(const hh_net* net, const LabelWindow& lw) {
  return net->nphase <= 4 && (net->n == 32 || net->n == 64) && rows_aligned(lw, net->n, 2);
}

// counts: label counts of the batch's input windows when the caller has them
// (the fraction features), else counted here into net->cnt; every launch on st
void forward_window(hh_ctx* ctx, hh_net* net, const LabelWindow& lw, int batch, const int* counts, hipStream_t st) {
  const int n = net->n;
  net->lw = lw;
  if (counts) {
    net->cnt_in = counts;
  } else {
    k_zero_int<<<(batch * kFrac + 255) / 256, 256, 0, st>>>(net->cnt, batch * kFrac);
    launch_count_labels(lw, n, 0, batch, net->cnt, st);
    net->cnt_in = net->cnt;
  }
  if (lw.mx > 0 && !staged_first_layer(net, lw)) fail(ctx, HH_EINVAL, "internal: image windows need the staged first layer");
  // labels of at most four phases: the four-channel paths (fewer k-steps);
  // the row path loads two labels at a time and needs every window row to
  // start on an even address
  auto aligned = [&](int w) { return rows_aligned(lw, n, w); };
  const int Do = n / 2, nvo = Do * Do * Do;
  const dim3 g1(unsigned((nvo + 255) / 256), unsigned(batch));
  const float* b0 = net->p + net->boff[0];
  if (net->nphase <= 4 && aligned(2)) {
    // output edges 16 and 32: the workgroup's labels and the weights staged in LDS
    const bool a8 = aligned(8);
    if (Do == 32 && a8)
      k_conv_fwd_rows4s<32, 8, 32><<<g1, 256, 0, st>>>(net->lw, net->WR, b0, net->a[0]);
    else if (Do == 32)
      k_conv_fwd_rows4s<32, 2, 32><<<g1, 256, 0, st>>>(net->lw, net->WR, b0, net->a[0]);
    else if (Do == 16 && a8)
      k_conv_fwd_rows4s<16, 8, 32><<<g1, 256, 0, st>>>(net->lw, net->WR, b0, net->a[0]);
    else if (Do == 16)
      k_conv_fwd_rows4s<16, 2, 32><<<g1, 256, 0, st>>>(net->lw, net->WR, b0, net->a[0]);
    else
      k_conv_fwd_rows4<32, 4><<<g1, 256, 0, st>>>(net->lw, net->WR, b0, net->a[0], make_grid3(Do));
  } else if (net->nphase <= 4)
    conv_fwd<4, 32, true, 4>(ctx, nullptr, net->lw, net->W4, net->p + net->boff[0], net->a[0], edge(net, 0), batch, st);
  else
    conv_fwd<8, 32, true, 4>(ctx, nullptr, net->lw, net->W[0], net->p + net->boff[0], net->a[0], edge(net, 0), batch, st);
  conv_fwd<32, 32, false, 4>(ctx, net->a[0], net->lw, net->W[1], net->p + net->boff[1], net->a[1], edge(net, 1), batch, st);
  conv_fwd<32, 64, false, 2>(ctx, net->a[1], net->lw, net->W[2], net->p + net->boff[2], net->a[2], edge(net, 2), batch, st);
  conv_fwd_splitk<64, 64>(ctx, net->a[2], net->W[3], net->p + net->boff[3], net->a[3], edge(net, 3), batch, st);
  HIPCHK(hipGetLastError());
}

// the windows at (o, o, o) of `batch` label boxes of edge box, back to back
void forward(hh_ctx* ctx, hh_net* net, const unsigned char* labels, int batch, int box, int o, const int* counts,
             hipStream_t st) {
  forward_window(ctx, net, box_window(labels, (long long)box * box * box, box, o), batch, counts, st);
}

// c21 (or null): the denormalized predictions, written by the head as well
void head(hh_ctx* ctx, hh_net* net, int batch, const float* target, float* dA, float* dW, float* loss, float inv,
          hipStream_t st, double* c21 = nullptr) {
  const int V = edge(net, 3) / 2;
  const double nv = double(net->n) * net->n * net->n;
  k_head<<<batch, 64, 0, st>>>(net->a[3], V * V * V, net->cnt_in, 1.0 / nv, net->d_fmu, net->d_fsc,
                                        net->p + net->fcw_off, net->p + net->fcb_off, net->out, target, dA, dW, loss,
                                        inv, net->d_mean, net->d_scale, c21);
}

template <int CI, int CO, bool LAB>
void conv_bwd(hh_ctx* ctx, hh_net* net, int l, const __bf16* X, int batch, float* dX) {
  const int D = edge(net, l), Do = D / 2;
  const long long total = (long long)Do * Do * Do * batch;
  const int chunk = wgrad_chunk(total, LAB ? kMaxChunksLab : kMaxChunks);
  const int nch = int((total + chunk - 1) / chunk);
  if (nch > (LAB ? kMaxChunksLab : kMaxChunks)) fail(ctx, HH_EINVAL, "internal: weight-gradient chunk count");
  if constexpr (LAB)
    k_conv_wgrad_lab<CO><<<nch, 256, 0, ctx->stream>>>(net->ga[l], net->a[l], net->lw, net->part, net->pbias,
                                                       make_grid3(D / 2), batch, chunk);
  else
    k_conv_wgrad<CI, CO><<<dim3(nch, 27), 256, 0, ctx->stream>>>(net->ga[l], net->a[l], X, net->part, net->pbias, D,
                                                                 make_grid3(D / 2), batch, chunk);
  const long long nw = 27LL * CO * CI;
  k_reduce_parts_wide<<<unsigned((nw + 63) / 64), 1024, 0, ctx->stream>>>(net->part, nch, nw,
                                                                          net->g + net->woff[l]);
  k_reduce_parts_wide<<<unsigned((CO + 63) / 64), 1024, 0, ctx->stream>>>(net->pbias, nch, CO,
                                                                          net->g + net->boff[l]);
  if constexpr (CI >= 16) {
    if (dX) {
      const int h = D / 2, ncls = h * h * h;  // voxels of one parity class per item
      for (int c = 0; c < 8; ++c)
        k_conv_dgrad<CI, CO><<<dim3(unsigned((ncls + 63) / 64), unsigned(batch)), 256, 0, ctx->stream>>>(
            net->ga[l], net->a[l], net->Wt[l], dX, D, make_grid3(h), c);
    }
  }
  HIPCHK(hipGetLastError());
}

// loss and gradient into net->g; returns the mean squared error
float backward(hh_ctx* ctx, hh_net* net, int batch) {
  const float inv = 1.0f / float(batch * kOut);
  head(ctx, net, batch, net->tgt, net->ga[3], net->hw, net->loss, inv, ctx->stream);
  k_reduce_parts<<<8, 256, 0, ctx->stream>>>(net->hw, batch, kOut * kFeat + kOut, net->g + net->fcw_off);
  conv_bwd<64, 64, false>(ctx, net, 3, net->a[2], batch, net->ga[2]);
  conv_bwd<32, 64, false>(ctx, net, 2, net->a[1], batch, net->ga[1]);
  conv_bwd<32, 32, false>(ctx, net, 1, net->a[0], batch, net->ga[0]);
  conv_bwd<8, 32, true>(ctx, net, 0, nullptr, batch, nullptr);
  std::vector<float> lh(batch);
  HIPCHK(hipMemcpyAsync(lh.data(), net->loss, sizeof(float) * batch, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double s = 0.0;
  for (float x : lh) s += x;
  return float(s);
}

const unsigned char* labels_to_device(hh_ctx* ctx, const uint8_t* labels, int on_device, long long bytes) {
  if (on_device) return labels;
  auto* d = static_cast<unsigned char*>(ws(ctx, "net_labels", size_t(bytes)));
  HIPCHK(hipMemcpyAsync(d, labels, size_t(bytes), hipMemcpyHostToDevice, ctx->stream));
  return d;
}

void upload_fraction_scaling(hh_ctx* ctx, hh_net* net) {
  float mu[kFrac], sc[kFrac];
  for (int i = 0; i < kFrac; ++i) {
    mu[i] = float(net->fmu[i]);
    sc[i] = float(net->fsc[i]);
  }
  HIPCHK(hipMemcpyAsync(net->d_fmu, mu, sizeof(mu), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(net->d_fsc, sc, sizeof(sc), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
}

void check_input(hh_ctx* ctx, hh_net* net, int batch, int box, int o) {
  if (!net) fail(ctx, HH_EINVAL, "null network");
  if (batch < 1 || batch > 65535) fail(ctx, HH_EINVAL, "batch must be in [1, 65535]");
  if (o < 0 || o + net->n > box) fail(ctx, HH_EINVAL, "input window outside the boxes");
}

}  // namespace

void hh_net_predict_device(hh_ctx* ctx, hh_net* net, const unsigned char* labels, int batch, int box, int o,
                           double* c21, const int* counts, hipStream_t st) {
  // items per forward pass: 512 fill the grids of the small deep layers
  // (256: 5 % slower end to end; 1024: no faster)
  const int step = 512;
  ensure_acts(ctx, net, std::min(step, batch));
  for (int b0 = 0; b0 < batch; b0 += step) {
    const int nb = std::min(step, batch - b0);
    forward(ctx, net, labels + (long long)b0 * box * box * box, nb, box, o,
            counts ? counts + (long long)b0 * kFrac : nullptr, st);
    head(ctx, net, nb, nullptr, nullptr, nullptr, nullptr, 0.0f, st, c21 + (long long)b0 * kOut);
    HIPCHK(hipGetLastError());
  }
}

bool hh_net_image_input(const hh_net* net, const unsigned char* img, int nx, int ny) {
  return net && staged_first_layer(net, image_window(img, nx, ny, net->n, 0));
}

void hh_net_predict_image(hh_ctx* ctx, hh_net* net, const unsigned char* img, int nx, int ny, int nitems,
                          double* c21, const int* counts, hipStream_t st, hipEvent_t counts_ready) {
  const int step = 512;  // as in hh_net_predict_device
  ensure_acts(ctx, net, std::min(step, nitems));
  for (int b0 = 0; b0 < nitems; b0 += step) {
    const int nb = std::min(step, nitems - b0);
    forward_window(ctx, net, image_window(img, nx, ny, net->n, b0), nb,
                   counts ? counts + (long long)b0 * kFrac : nullptr, st);
    if (b0 == 0 && counts_ready) HIPCHK(hipStreamWaitEvent(st, counts_ready, 0));
    head(ctx, net, nb, nullptr, nullptr, nullptr, nullptr, 0.0f, st, c21 + (long long)b0 * kOut);
    HIPCHK(hipGetLastError());
  }
}

void hh_launch_counts(const unsigned char* labels, int nitems, int box, int o, int n, int* counts, hipStream_t st) {
  k_zero_int<<<(nitems * 8 + 255) / 256, 256, 0, st>>>(counts, nitems * 8);
  launch_count_labels(box_window(labels, (long long)box * box * box, box, o), n, 0, nitems, counts, st);
}

void hh_launch_counts_image(const unsigned char* img, int nx, int ny, int n, int nitems, int* counts,
                            hipStream_t st) {
  k_zero_int<<<(nitems * 8 + 255) / 256, 256, 0, st>>>(counts, nitems * 8);
  launch_count_labels(image_window(img, nx, ny, n, 0), n, 0, nitems, counts, st);
}

void hh_launch_bounds(const int* counts, int nitems, int n, int nphase, const double* Cp21, const double* Sp21,
                      double* cv21, double* cr21, hipStream_t st) {
  k_bounds_from_counts<<<(nitems + 63) / 64, 64, 0, st>>>(counts, nitems, 1.0 / (double(n) * n * n), nphase, Cp21,
                                                          Sp21, cv21, cr21);
}

void hh_launch_gate(const double* c21a, const double* c21b, const double* cv21, const double* cr21, int nitems,
                    double spread_tol, double bound_tol, const FracGate& ga, const FracGate& gb, int* flag,
                    hipStream_t st) {
  k_gate<<<(nitems + 63) / 64, 64, 0, st>>>(c21a, c21b, cv21, cr21, nitems, spread_tol, bound_tol, ga, gb, flag);
}

FracGate hh_net_fraction_gate(const hh_net* net, const int* counts, const unsigned* iface) {
  FracGate q;
  if (!net) return q;
  q.counts = counts;
  q.inv_nv = 1.0 / (double(net->n) * net->n * net->n);
  for (int c = 0; c < kFrac; ++c) {
    q.mu[c] = net->fmu[c];
    q.sc[c] = net->fsc[c];
  }
  q.zmax = net->fzmax;
  if (net->isc > 0.0 && iface) {
    q.iface = iface;
    q.inv_pairs = 1.0 / (3.0 * double(net->n) * net->n * (net->n - 1));
    q.imu = net->imu;
    q.isc = net->isc;
  }
  return q;
}

bool hh_net_has_interface_stats(const hh_net* net) { return net && net->isc > 0.0 && net->n > 1; }

void hh_launch_interfaces(const unsigned char* labels, int nitems, int box, int o, int n, unsigned* counts,
                          hipStream_t st) {
  k_zero_int<<<(nitems + 255) / 256, 256, 0, st>>>(reinterpret_cast<int*>(counts), nitems);
  launch_count_interfaces(box_window(labels, (long long)box * box * box, box, o), n, 0, nitems, counts, st);
}

void hh_launch_interfaces_image(const unsigned char* img, int nx, int ny, int n, int nitems, unsigned* counts,
                                hipStream_t st, int* label_counts) {
  k_zero_int<<<(nitems + 255) / 256, 256, 0, st>>>(reinterpret_cast<int*>(counts), nitems);
  if (label_counts) k_zero_int<<<(nitems * 8 + 255) / 256, 256, 0, st>>>(label_counts, nitems * 8);
  launch_count_interfaces(image_window(img, nx, ny, n, 0), n, 0, nitems, counts, st, label_counts);
}

int hh_net_input_size(const hh_net* net) { return net ? net->n : 0; }

extern "C" {

int hh_net_create(hh_ctx* ctx, int nphase, int n, unsigned long long seed, hh_net** out) {
  return guarded(ctx, [&]() -> int {
    if (!out) fail(ctx, HH_EINVAL, "null output");
    *out = nullptr;
    if (nphase < 1 || nphase > 8) fail(ctx, HH_EINVAL, "the surrogate takes 1..8 phases");
    if (n < 16 || n % 16 != 0 || n > 256) fail(ctx, HH_EINVAL, "input edge must be a multiple of 16 in [16, 256]");
    auto* net = new hh_net();
    net->device = ctx->device;
    net->nphase = nphase;
    net->n = n;
    long long off = 0;
    for (int l = 0; l < kLayers; ++l) {
      net->woff[l] = off;
      off += 27LL * kCout[l] * kCin[l];
      net->boff[l] = off;
      off += kCout[l];
    }
    net->fcw_off = off;
    off += kOut * kFeat;
    net->fcb_off = off;
    off += kOut;
    net->nparam = off;
    try {
      net->p = dalloc<float>(ctx, off);
      net->g = dalloc<float>(ctx, off);
      net->m = dalloc<float>(ctx, off);
      net->v = dalloc<float>(ctx, off);
      for (int l = 0; l < kLayers; ++l) {
        net->W[l] = dalloc<__bf16>(ctx, 27LL * kCout[l] * kCin[l]);
        net->Wt[l] = dalloc<__bf16>(ctx, 27LL * kCout[l] * kCin[l]);
      }
      net->W4 = dalloc<__bf16>(ctx, 14LL * kCout[0] * 8);
      net->WR = dalloc<__bf16>(ctx, 20LL * kCout[0] * 8);
      net->d_mean = dalloc<double>(ctx, kOut);
      net->d_scale = dalloc<double>(ctx, kOut);
      net->d_fmu = dalloc<float>(ctx, kFrac);
      net->d_fsc = dalloc<float>(ctx, kFrac);
    } catch (...) {
      hh_net_destroy(net);
      throw;
    }
    // He initialisation (fan-in of the real input channels); padded input
    // channels of the first layer start (and stay) at zero
    std::vector<float> h(off, 0.0f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < kLayers; ++l) {
      const int cin_real = l == 0 ? nphase : kCin[l];
      std::normal_distribution<float> nd(0.0f, std::sqrt(2.0f / (27.0f * cin_real)));
      for (int t = 0; t < 27; ++t)
        for (int co = 0; co < kCout[l]; ++co)
          for (int ci = 0; ci < kCin[l]; ++ci)
            h[net->woff[l] + ((long long)t * kCout[l] + co) * kCin[l] + ci] = ci < cin_real ? nd(rng) : 0.0f;
    }
    std::normal_distribution<float> nf(0.0f, std::sqrt(1.0f / kFeat));
    for (int i = 0; i < kOut * kFeat; ++i) h[net->fcw_off + i] = nf(rng);
    for (int i = 0; i < kOut; ++i) {
      net->mean[i] = 0.0;
      net->scale[i] = 1.0;
    }
    for (int i = 0; i < kFrac; ++i) {
      net->fmu[i] = 0.0;
      net->fsc[i] = 1.0;
    }
    upload_fraction_scaling(ctx, net);
    HIPCHK(hipMemcpyAsync(net->p, h.data(), sizeof(float) * off, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemsetAsync(net->m, 0, sizeof(float) * off, ctx->stream));
    HIPCHK(hipMemsetAsync(net->v, 0, sizeof(float) * off, ctx->stream));
    HIPCHK(hipMemcpyAsync(net->d_mean, net->mean, sizeof(double) * kOut, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(net->d_scale, net->scale, sizeof(double) * kOut, hipMemcpyHostToDevice, ctx->stream));
    cast_all(ctx, net);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = net;
    return HH_OK;
  });
}

void hh_net_destroy(hh_net* net) {
  if (!net) return;
  (void)hipSetDevice(net->device);
  (void)hipDeviceSynchronize();
  free_acts(net);
  (void)hipFree(net->p);
  (void)hipFree(net->g);
  (void)hipFree(net->m);
  (void)hipFree(net->v);
  for (int l = 0; l < kLayers; ++l) {
    (void)hipFree(net->W[l]);
    (void)hipFree(net->Wt[l]);
    if (l == 0) {
      (void)hipFree(net->W4);
      (void)hipFree(net->WR);
    }
  }
  (void)hipFree(net->d_mean);
  (void)hipFree(net->d_scale);
  (void)hipFree(net->d_fmu);
  (void)hipFree(net->d_fsc);
  delete net;
}

long long hh_net_num_params(const hh_net* net) { return net ? net->nparam : 0; }

int hh_net_get_params(hh_ctx* ctx, hh_net* net, float* params, long long n) {
  return guarded(ctx, [&]() -> int {
    if (!net || !params || n != net->nparam) fail(ctx, HH_EINVAL, "parameter count mismatch");
    HIPCHK(hipMemcpyAsync(params, net->p, sizeof(float) * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return HH_OK;
  });
}

int hh_net_set_params(hh_ctx* ctx, hh_net* net, const float* params, long long n) {
  return guarded(ctx, [&]() -> int {
    if (!net || !params || n != net->nparam) fail(ctx, HH_EINVAL, "parameter count mismatch");
    HIPCHK(hipMemcpyAsync(net->p, params, sizeof(float) * n, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemsetAsync(net->m, 0, sizeof(float) * n, ctx->stream));
    HIPCHK(hipMemsetAsync(net->v, 0, sizeof(float) * n, ctx->stream));
    net->step = 0;
    cast_all(ctx, net);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return HH_OK;
  });
}

int hh_net_set_scaling(hh_ctx* ctx, hh_net* net, const double mean[21], const double scale[21]) {
  return guarded(ctx, [&]() -> int {
    if (!net || !mean || !scale) fail(ctx, HH_EINVAL, "null argument");
    for (int i = 0; i < kOut; ++i) {
      if (!(scale[i] > 0.0) || !std::isfinite(mean[i])) fail(ctx, HH_EINVAL, "scales must be positive");
      net->mean[i] = mean[i];
      net->scale[i] = scale[i];
    }
    HIPCHK(hipMemcpyAsync(net->d_mean, net->mean, sizeof(double) * kOut, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(net->d_scale, net->scale, sizeof(double) * kOut, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return HH_OK;
  });
}

int hh_net_set_fraction_scaling(hh_ctx* ctx, hh_net* net, const double mean[8], const double scale[8]) {
  return guarded(ctx, [&]() -> int {
    if (!net || !mean || !scale) fail(ctx, HH_EINVAL, "null argument");
    for (int i = 0; i < kFrac; ++i)
      if (!std::isfinite(mean[i]) || !std::isfinite(scale[i])) fail(ctx, HH_EINVAL, "non-finite scaling");
    for (int i = 0; i < kFrac; ++i) {
      net->fmu[i] = mean[i];
      net->fsc[i] = scale[i];
    }
    upload_fraction_scaling(ctx, net);
    return HH_OK;
  });
}

int hh_net_set_fraction_gate(hh_ctx* ctx, hh_net* net, double z_max) {
  return guarded(ctx, [&]() -> int {
    if (!net) fail(ctx, HH_EINVAL, "null network");
    if (!std::isfinite(z_max) || z_max < 0.0) fail(ctx, HH_EINVAL, "z_max must be finite and >= 0");
    net->fzmax = z_max;
    return HH_OK;
  });
}

int hh_net_set_interface_stats(hh_ctx* ctx, hh_net* net, double mean, double scale) {
  return guarded(ctx, [&]() -> int {
    if (!net) fail(ctx, HH_EINVAL, "null network");
    if (!std::isfinite(mean) || !std::isfinite(scale) || mean < 0.0 || mean > 1.0 || scale < 0.0)
      fail(ctx, HH_EINVAL, "interface statistics: mean in [0, 1] and a finite scale >= 0");
    net->imu = mean;
    net->isc = scale;
    return HH_OK;
  });
}

int hh_net_get_interface_stats(const hh_net* net, double* mean, double* scale) {
  if (!net || !mean || !scale) return HH_EINVAL;
  *mean = net->imu;
  *scale = net->isc;
  return HH_OK;
}

int hh_net_get_fraction_scaling(const hh_net* net, double mean[8], double scale[8]) {
  if (!net || !mean || !scale) return HH_EINVAL;
  for (int i = 0; i < kFrac; ++i) {
    mean[i] = net->fmu[i];
    scale[i] = net->fsc[i];
  }
  return HH_OK;
}

int hh_net_info(const hh_net* net, int* nphase, int* n) {
  if (!net || !nphase || !n) return HH_EINVAL;
  *nphase = net->nphase;
  *n = net->n;
  return HH_OK;
}

int hh_net_get_scaling(const hh_net* net, double mean[21], double scale[21]) {
  if (!net || !mean || !scale) return HH_EINVAL;
  for (int i = 0; i < kOut; ++i) {
    mean[i] = net->mean[i];
    scale[i] = net->scale[i];
  }
  return HH_OK;
}

int hh_net_forward(hh_ctx* ctx, hh_net* net, const uint8_t* labels, int labels_on_device, int batch, int box,
                   int offset, float* out) {
  return guarded(ctx, [&]() -> int {
    check_input(ctx, net, batch, box, offset);
    if (!labels || !out) fail(ctx, HH_EINVAL, "null argument");
    const unsigned char* d = labels_to_device(ctx, labels, labels_on_device, (long long)batch * box * box * box);
    ensure_acts(ctx, net, batch);
    forward(ctx, net, d, batch, box, offset, nullptr, ctx->stream);
    head(ctx, net, batch, nullptr, nullptr, nullptr, nullptr, 0.0f, ctx->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, net->out, sizeof(float) * batch * kOut, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return HH_OK;
  });
}

int hh_net_gradient(hh_ctx* ctx, hh_net* net, const uint8_t* labels, int labels_on_device, int batch, int box,
                    int offset, const float* target, float* loss, float* grad) {
  return guarded(ctx, [&]() -> int {
    check_input(ctx, net, batch, box, offset);
    if (!labels || !target) fail(ctx, HH_EINVAL, "null argument");
    const unsigned char* d = labels_to_device(ctx, labels, labels_on_device, (long long)batch * box * box * box);
    ensure_acts(ctx, net, batch);
    HIPCHK(hipMemcpyAsync(net->tgt, target, sizeof(float) * batch * kOut, hipMemcpyHostToDevice, ctx->stream));
    forward(ctx, net, d, batch, box, offset, nullptr, ctx->stream);
    const float l = backward(ctx, net, batch);
    if (loss) *loss = l;
    if (grad) {
      HIPCHK(hipMemcpyAsync(grad, net->g, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return HH_OK;
  });
}

int hh_net_train_step(hh_ctx* ctx, hh_net* net, const uint8_t* labels, int labels_on_device, int batch, int box,
                      int offset, const float* target, int target_on_device, float lr, float* loss) {
  return guarded(ctx, [&]() -> int {
    check_input(ctx, net, batch, box, offset);
    if (!labels || !target || !(lr > 0.0f)) fail(ctx, HH_EINVAL, "bad argument");
    const unsigned char* d = labels_to_device(ctx, labels, labels_on_device, (long long)batch * box * box * box);
    ensure_acts(ctx, net, batch);
    HIPCHK(hipMemcpyAsync(net->tgt, target, sizeof(float) * batch * kOut,
                          target_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
    forward(ctx, net, d, batch, box, offset, nullptr, ctx->stream);
    const float l = backward(ctx, net, batch);
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, float(net->step)), c2 = 1.0f - std::pow(b2, float(net->step));
    k_adam<<<unsigned(std::min<long long>((net->nparam + 255) / 256, 4096)), 256, 0, ctx->stream>>>(
        net->p, net->g, net->m, net->v, net->nparam, lr, b1, b2, 1e-8f, c1, c2);
    cast_all(ctx, net);
    if (loss) *loss = l;
    return HH_OK;
  });
}

int hh_net_predict(hh_ctx* ctx, hh_net* net, const uint8_t* labels, int labels_on_device, int batch, int box,
                   int offset, double* C21) {
  return guarded(ctx, [&]() -> int {
    check_input(ctx, net, batch, box, offset);
    if (!labels || !C21) fail(ctx, HH_EINVAL, "null argument");
    const unsigned char* d = labels_to_device(ctx, labels, labels_on_device, (long long)batch * box * box * box);
    auto* c = static_cast<double*>(ws(ctx, "net_c21", sizeof(double) * batch * kOut));
    hh_net_predict_device(ctx, net, d, batch, box, offset, c, nullptr, ctx->stream);
    HIPCHK(hipMemcpyAsync(C21, c, sizeof(double) * batch * kOut, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return HH_OK;
  });
}

}  // extern "C"

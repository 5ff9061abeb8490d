// FP64 finalize kernels of the solve (alpha, beta, convergence control),
// the stiffness C_R = Sigma E^-1 per item, and the size dispatcher.
#include "solver_kernels.hpp"

namespace hh {

// ---------------------------------------------------------------------------
// finalize kernels: one block per system, fixed-order FP64 reductions
// ---------------------------------------------------------------------------
// Sum of the per-workgroup partials of one system: each thread runs a
// Neumaier-compensated sum over its strided share (the running sum and the
// rounding error lost at each step, added back at the end), then a fixed
// tree over the block.
template <int NV>
__device__ __forceinline__ void reduce_parts(const double* part, int n, double (&v)[NV], double* scratch) {
  double comp[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    v[i] = 0.0;
    comp[i] = 0.0;
  }
  for (int w = threadIdx.x; w < n; w += blockDim.x) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double x = part[(long long)w * NV + i];
      const double t = v[i] + x;
      comp[i] += fabs(v[i]) >= fabs(x) ? (v[i] - t) + x : (x - t) + v[i];
      v[i] = t;
    }
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] += comp[i];
  block_sum<NV>(v, scratch);
}

// First stage of a finalize: block (c, s) sums the per-row (x) or
// per-column (z) values [c kFinChunk, (c + 1) kFinChunk) of system s; thread
// t takes every 256th one from t in order, then the block tree.  Systems
// that stopped are skipped except when the right-hand side is formed.
template <int NV>
__global__ void __launch_bounds__(256) k_fin_chunks(GroupArgs g, int rhs) {
  __shared__ double scratch[4 * NV];
  const int s = blockIdx.y;
  if (!rhs && g.state[s].status != kRunning) return;
  const bool x = NV == kPartX;
  const long long n = x ? g.nrow_x : g.ncol_z;
  const double* part = (x ? g.part_x : g.part_z) + (long long)s * n * NV;
  const long long i0 = (long long)blockIdx.x * kFinChunk, i1 = min(n, i0 + kFinChunk);
  double v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0.0;
  for (long long r = i0 + threadIdx.x; r < i1; r += 256) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += part[r * NV + i];
  }
  block_sum<NV>(v, scratch);
  if (threadIdx.x == 0) {
    double* out = (x ? g.chunk_x : g.chunk_z) + ((long long)s * gridDim.x + blockIdx.x) * NV;
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = v[i];
  }
}

__global__ void __launch_bounds__(256) k_fin_x(GroupArgs g, int mode) {
  __shared__ double scratch[4 * kPartX];
  const int s = blockIdx.x;
  SysState* st = g.state + s;
  if (mode != kXRhs && st->status != kRunning) return;
  double v[kPartX];
  reduce_parts<kPartX>(g.chunk_x + (long long)s * g.nchunk_x * kPartX, g.nchunk_x, v, scratch);
  if (threadIdx.x != 0) return;
  const ItemDesc& it = g.items[g.sys[s].item];
  const double inv = it.inv_region;
  if (mode == kXRhs) {
    for (int c = 0; c < 6; ++c) {
      st->sig[c] = v[7 + c] * inv;
      st->eps[c] = g.loads[g.sys[s].load][c];
    }
    for (int c = 0; c < 6; ++c) {
      st->sig_best[c] = st->sig[c];
      st->eps_best[c] = st->eps[c];
    }
    st->ce2 = v[0];
    st->bb = 0.0;
    st->rr = 0.0;
    st->best_rr = 1e300;
    st->status = kRunning;
    st->iter = 0;
    st->stall = 0;
    st->alpha = 0.0;
    st->beta = 0.0;
  } else if (mode == kXCg) {
    const double pap = v[0];
    if (!isfinite(pap)) {
      st->status = kNonFinite;
      return;
    }
    if (!(pap > 0.0)) {
      st->status = kBreakdown;
      return;
    }
    const double a = st->rr / pap;
    st->alpha = a;
    for (int c = 0; c < 6; ++c) {
      st->eps[c] += a * v[1 + c] * inv;
      st->sig[c] += a * v[7 + c] * inv;
    }
  } else {  // fixed point: averages of the current iterate
    for (int c = 0; c < 6; ++c) {
      st->eps[c] = v[1 + c] * inv;
      st->sig[c] = v[7 + c] * inv;
    }
  }
}

__global__ void __launch_bounds__(256) k_fin_z(GroupArgs g, int mode) {
  __shared__ double scratch[4];
  const int s = blockIdx.x;
  SysState* st = g.state + s;
  if (st->status != kRunning) return;
  double v[1];
  reduce_parts<1>(g.chunk_z + (long long)s * g.nchunk_z, g.nchunk_z, v, scratch);
  if (threadIdx.x != 0) return;
  const double V = double(g.nx) * g.ny * g.nz;
  const double rr = v[0] / V;
  if (!isfinite(rr)) {
    st->status = kNonFinite;
    return;
  }
  if (mode == kZFwdRhs || (mode == kZFwdFp && st->iter == 0)) {
    st->bb = rr;
    st->rr = rr;
    st->best_rr = rr;
    st->beta = 0.0;
    if (rr <= g.zero_rhs2 * st->ce2) {
      st->status = kConverged;
      return;
    }
    if (mode == kZFwdRhs) return;
  }
  const double prev = st->rr;
  st->rr = rr;
  if (mode == kZFwdCg) {
    st->beta = rr / prev;
    st->iter += 1;
  }
  if (rr < st->best_rr) {
    st->best_rr = rr;
    st->stall = 0;
    for (int c = 0; c < 6; ++c) {
      st->sig_best[c] = st->sig[c];
      st->eps_best[c] = st->eps[c];
    }
  } else {
    st->stall += 1;
  }
  if (rr <= g.tol2 * st->bb) {
    st->status = kConverged;
  } else if (st->stall >= g.stall_limit || rr > 1e4 * st->best_rr) {
    st->status = kStagnated;  // FP32 floor or divergence: keep the best iterate
  } else if (st->iter >= g.max_iter) {
    st->status = kNoConv;
  }
  if (st->status == kStagnated || st->status == kNoConv) {
    for (int c = 0; c < 6; ++c) {
      st->sig[c] = st->sig_best[c];
      st->eps[c] = st->eps_best[c];
    }
    st->rr = st->best_rr;
  }
  if (mode == kZFwdFp && st->status == kRunning) st->iter += 1;
}

// C_R = Sigma E^-1 per item (systems item*6 + a), FP64 Gauss-Jordan with
// partial pivoting on E^T C^T = Sigma^T.  out[item][0..36) raw, [36..72) sym.
// When cfield_out is set, also writes the symmetric 21 components per item
// as the stiffness field of the next level.
template <class T>
__global__ void k_stiffness(const SysState* state, int nitems, double* out, T* cfield_out,
                            int* status_out) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= nitems) return;
  double A[6][6], B[6][6];  // A = E^T, B = Sigma^T
  int worst = kConverged;
  for (int a = 0; a < 6; ++a) {
    const SysState& st = state[item * 6 + a];
    if (st.status != kConverged && worst == kConverged) worst = st.status;
    for (int c = 0; c < 6; ++c) {
      A[a][c] = st.eps[c] * (c < 3 ? 1.0 : 2.0);
      B[a][c] = st.sig[c];
    }
  }
  int singular = 0;
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    double best = fabs(A[col][col]);
    for (int r = col + 1; r < 6; ++r)
      if (fabs(A[r][col]) > best) {
        best = fabs(A[r][col]);
        piv = r;
      }
    if (!(best > 1e-300)) {
      singular = 1;
      break;
    }
    if (piv != col)
      for (int c = 0; c < 6; ++c) {
        double t = A[col][c];
        A[col][c] = A[piv][c];
        A[piv][c] = t;
        t = B[col][c];
        B[col][c] = B[piv][c];
        B[piv][c] = t;
      }
    const double d = 1.0 / A[col][col];
    for (int c = 0; c < 6; ++c) {
      A[col][c] *= d;
      B[col][c] *= d;
    }
    for (int r = 0; r < 6; ++r) {
      if (r == col) continue;
      const double f = A[r][col];
      if (f == 0.0) continue;
      for (int c = 0; c < 6; ++c) {
        A[r][c] -= f * A[col][c];
        B[r][c] -= f * B[col][c];
      }
    }
  }
  double* o = out + (long long)item * 72;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      const double cij = singular ? 0.0 : B[j][i];  // C = (E^T)^-1 Sigma^T transposed
      o[i * 6 + j] = cij;
    }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) o[36 + i * 6 + j] = 0.5 * (o[i * 6 + j] + o[j * 6 + i]);
  if (cfield_out) {
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i; j < 6; ++j) cfield_out[(long long)item * 21 + k++] = T(o[36 + i * 6 + j]);
  }
  if (status_out) status_out[item] = singular ? kSingularStatus : worst;
}

SizeOpsFn size_ops(int n, int precision, int variant) {
  using Part = SizeOpsFn (*)(int, int);
  if (variant < 0 || variant >= kNVariant) return nullptr;
  static const Part f32[] = {size_ops_f32_0, size_ops_f32_1, size_ops_f32_2, size_ops_f32_3, size_ops_f32_4, size_ops_f32_5, size_ops_f32_6, size_ops_f32_7, size_ops_f32_8, size_ops_f32_9, size_ops_f32_10, size_ops_f32_11, size_ops_f32_12, size_ops_f32_13, size_ops_f32_14, size_ops_f32_15, size_ops_f32_16, size_ops_f32_17, size_ops_f32_18, size_ops_f32_19, size_ops_f32_20, size_ops_f32_21, size_ops_f32_22, size_ops_f32_23, size_ops_f32_24, size_ops_f32_25, size_ops_f32_26, size_ops_f32_27, size_ops_f32_28};
  static const Part f64[] = {size_ops_f64_0, size_ops_f64_1, size_ops_f64_2, size_ops_f64_3,
                             size_ops_f64_4, size_ops_f64_5, size_ops_f64_6};
  if (precision == 0) {
    for (Part p : f32)
      if (SizeOpsFn f = p(n, variant)) return f;
  } else if (precision == 1) {
    for (Part p : f64)
      if (SizeOpsFn f = p(n, variant)) return f;
  }
  return nullptr;
}

void launch_fin_x(int mode, const GroupArgs& g, hipStream_t st) {
  k_fin_chunks<kPartX><<<dim3(g.nchunk_x, g.nsys), 256, 0, st>>>(g, mode == kXRhs ? 1 : 0);
  k_fin_x<<<g.nsys, 256, 0, st>>>(g, mode);
}
void launch_fin_z(int mode, const GroupArgs& g, hipStream_t st) {
  k_fin_chunks<1><<<dim3(g.nchunk_z, g.nsys), 256, 0, st>>>(g, mode == kZFwdRhs ? 1 : 0);
  k_fin_z<<<g.nsys, 256, 0, st>>>(g, mode);
}
void launch_stiffness(int precision, const SysState* state, int nitems, double* out, void* cfield_out,
                      int* status_out, hipStream_t st) {
  const int b = 64, nb = (nitems + b - 1) / b;
  if (precision == 0)
    k_stiffness<float><<<nb, b, 0, st>>>(state, nitems, out, reinterpret_cast<float*>(cfield_out), status_out);
  else
    k_stiffness<double><<<nb, b, 0, st>>>(state, nitems, out, reinterpret_cast<double*>(cfield_out), status_out);
}

}  // namespace hh

// Restarted GMRES kernels for (sigma I + Z^F) x = b, with nrhs independent
// right-hand sides sharing each far-zone product launch.
//
// Krylov vectors are complex64 (the product's input format); every inner
// product, norm, Gram-Schmidt update and the Hessenberg / Givens / least-
// squares state are FP64. Reductions are two-level with a fixed block count
// and a fixed summation order, so results repeat bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gmres.hpp"

namespace ubf {
namespace {

constexpr int kThreads = 256;
constexpr int kColTile = 8;  // Krylov columns per pass over w

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ inline double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 f2d(float2 v) { return make_double2(v.x, v.y); }

// Block-wide sum of one double2 per thread; result valid in thread 0.
__device__ double2 block_sum(double2 v, double2* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_down(v.x, o, 64);
    v.y += __shfl_down(v.y, o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) {
      s.x += sh[w].x;
      s.y += sh[w].y;
    }
  return s;
}

// partial[(blk * R + r) * ldp + c] = sum over this block's slice of
// conj(V_c[r][i]) * w[r][i], for columns c < ncol. V_c = V + c * vstride.
__global__ __launch_bounds__(kThreads) void dots_kernel(
    const float2* __restrict__ V, int64_t vstride, int ncol, const float2* __restrict__ w,
    int64_t n, int R, double2* __restrict__ partial, int ldp) {
  __shared__ double2 sh[kThreads / 64];
  const int r = blockIdx.y;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  const float2* wr = w + (int64_t)r * n;
  for (int c0 = 0; c0 < ncol; c0 += kColTile) {
    double2 acc[kColTile];
#pragma unroll
    for (int t = 0; t < kColTile; ++t) acc[t] = make_double2(0.0, 0.0);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
      const double2 wv = f2d(wr[i]);
#pragma unroll
      for (int t = 0; t < kColTile; ++t)
        if (c0 + t < ncol) {
          const double2 p = cmulc(f2d(V[(int64_t)(c0 + t) * vstride + (int64_t)r * n + i]), wv);
          acc[t].x += p.x;
          acc[t].y += p.y;
        }
    }
#pragma unroll
    for (int t = 0; t < kColTile; ++t) {
      if (c0 + t >= ncol) break;  // uniform
      const double2 s = block_sum(acc[t], sh);
      if (threadIdx.x == 0)
        partial[((int64_t)blockIdx.x * R + r) * ldp + c0 + t] = s;
    }
  }
}

// out[r * ldo + c] = sum over blocks (in block order) of the partials.
__global__ __launch_bounds__(64) void reduce_kernel(const double2* __restrict__ partial,
                                                    int nblk, int R, int ncol, int ldp,
                                                    double2* __restrict__ out, int ldo) {
  const int r = blockIdx.x;
  for (int c = threadIdx.x; c < ncol; c += 64) {
    double2 s = make_double2(0.0, 0.0);
    for (int b = 0; b < nblk; ++b) {
      const double2 p = partial[((int64_t)b * R + r) * ldp + c];
      s.x += p.x;
      s.y += p.y;
    }
    out[(int64_t)r * ldo + c] = s;
  }
}

// w[r][i] -= sum_c V_c[r][i] * h[r][c]  (FP64 sum, one rounding to FP32).
__global__ __launch_bounds__(kThreads) void update_kernel(
    const float2* __restrict__ V, int64_t vstride, int ncol, const double2* __restrict__ h,
    int ldh, float2* __restrict__ w, int64_t n, int R) {
  __shared__ double2 hs[kMaxRestart + 1];
  const int r = blockIdx.y;
  for (int c = threadIdx.x; c < ncol; c += kThreads) hs[c] = h[(int64_t)r * ldh + c];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    double2 s = f2d(w[(int64_t)r * n + i]);
    for (int c = 0; c < ncol; ++c) {
      const double2 p = cmul(f2d(V[(int64_t)c * vstride + (int64_t)r * n + i]), hs[c]);
      s.x -= p.x;
      s.y -= p.y;
    }
    w[(int64_t)r * n + i] = make_float2((float)s.x, (float)s.y);
  }
}

// w += sigma * v
__global__ __launch_bounds__(kThreads) void add_shift_kernel(float2* __restrict__ w,
                                                             const float2* __restrict__ v,
                                                             double sr, double si, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    const double2 a = f2d(w[i]), b = f2d(v[i]);
    w[i] = make_float2((float)(a.x + sr * b.x - si * b.y), (float)(a.y + sr * b.y + si * b.x));
  }
}

// dst[r][i] = src[r][i] * s[r]  (real per-RHS scale)
__global__ __launch_bounds__(kThreads) void scale_kernel(float2* __restrict__ dst,
                                                         const float2* __restrict__ src,
                                                         const double* __restrict__ s,
                                                         int64_t n, int R) {
  const int r = blockIdx.y;
  const double f = s[r];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const float2 v = src[(int64_t)r * n + i];
    dst[(int64_t)r * n + i] = make_float2((float)(v.x * f), (float)(v.y * f));
  }
}

// dst = b - sigma x - ax  (residual of the shifted system)
__global__ __launch_bounds__(kThreads) void residual_kernel(float2* __restrict__ dst,
                                                            const float2* __restrict__ b,
                                                            const float2* __restrict__ x,
                                                            const float2* __restrict__ ax,
                                                            double sr, double si, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    const double2 bv = f2d(b[i]), xv = f2d(x[i]), av = f2d(ax[i]);
    dst[i] = make_float2((float)(bv.x - (sr * xv.x - si * xv.y) - av.x),
                         (float)(bv.y - (sr * xv.y + si * xv.x) - av.y));
  }
}

// Start of a cycle: beta = ||r|| (nrm[r].x = sum |r_i|^2). For the first
// cycle the norm is also ||b||. Sets g = (beta, 0, ...), the scale 1/beta
// of V_0, and deactivates right-hand sides already within tolerance.
__global__ void cycle_start_kernel(GmresState st, int R, int first, double tol) {
  const int r = threadIdx.x;
  if (r >= R) return;
  const double beta = sqrt(st.nrm[r].x);
  if (first) {
    st.bnorm[r] = beta;
    st.active[r] = 1;
    st.iters[r] = 0;
    st.res[r] = beta > 0.0 ? 1.0 : 0.0;
  }
  st.k[r] = 0;
  for (int i = 0; i <= st.m; ++i) st.g[r * (st.m + 1) + i] = make_double2(0.0, 0.0);
  const double bn = st.bnorm[r];
  const double rel = bn > 0.0 ? beta / bn : 0.0;
  if (st.active[r] && (beta == 0.0 || rel <= tol)) {
    st.active[r] = 0;
    st.res[r] = rel;
  }
  if (st.active[r]) {
    st.res[r] = rel;
    st.g[r * (st.m + 1)] = make_double2(beta, 0.0);
    st.scale[r] = 1.0 / beta;
  } else {
    st.scale[r] = 0.0;
  }
}

// Arnoldi column j: h = h1 + h2 (two Gram-Schmidt passes), h_{j+1,j} =
// ||w||; apply the earlier Givens rotations, make the new one, update the
// least-squares right-hand side g and the residual estimate |g_{j+1}|.
__global__ void arnoldi_tail_kernel(GmresState st, int R, int j, double tol) {
  const int r = threadIdx.x;
  if (r >= R) return;
  const int m = st.m, ld = m + 1;
  if (!st.active[r]) {
    st.scale[r] = 0.0;
    return;
  }
  double2* Hc = st.H + ((int64_t)r * m + j) * ld;  // column j of rhs r
  double colnorm2 = 0.0;
  for (int i = 0; i <= j; ++i) {
    const double2 a = st.h1[r * ld + i], b = st.h2[r * ld + i];
    Hc[i] = make_double2(a.x + b.x, a.y + b.y);
    colnorm2 += Hc[i].x * Hc[i].x + Hc[i].y * Hc[i].y;
  }
  const double hn = sqrt(st.nrm[r].x);
  // earlier rotations: [x; y] <- [c x + s y; -conj(s) x + c y]
  for (int i = 0; i < j; ++i) {
    const double c = st.cs[r * m + i];
    const double2 s = st.sn[r * m + i];
    const double2 x = Hc[i], y = Hc[i + 1];
    const double2 sy = cmul(s, y), sx = cmulc(s, x);
    Hc[i] = make_double2(c * x.x + sy.x, c * x.y + sy.y);
    Hc[i + 1] = make_double2(-sx.x + c * y.x, -sx.y + c * y.y);
  }
  // new rotation zeroing hn below a = Hc[j]
  const double2 a = Hc[j];
  const double aa = sqrt(a.x * a.x + a.y * a.y);
  double c;
  double2 s;
  if (hn == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    s = make_double2(1.0, 0.0);
  } else {
    const double t = sqrt(aa * aa + hn * hn);
    c = aa / t;
    s = make_double2(a.x / aa * hn / t, a.y / aa * hn / t);
  }
  st.cs[r * m + j] = c;
  st.sn[r * m + j] = s;
  {
    const double t = sqrt(aa * aa + hn * hn);
    Hc[j] = aa == 0.0 ? make_double2(hn, 0.0) : make_double2(a.x / aa * t, a.y / aa * t);
  }
  Hc[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = st.g[r * ld + j];
  const double2 sg = cmulc(s, gj);
  st.g[r * ld + j] = make_double2(c * gj.x, c * gj.y);
  st.g[r * ld + j + 1] = make_double2(-sg.x, -sg.y);
  st.k[r] = j + 1;
  st.iters[r] += 1;
  const double2 gn = st.g[r * ld + j + 1];
  const double rel = sqrt(gn.x * gn.x + gn.y * gn.y) / st.bnorm[r];
  st.res[r] = rel;
  // lucky breakdown (the Krylov space is invariant) or convergence
  const bool broke = hn <= 1e-14 * sqrt(colnorm2 + hn * hn);
  if (rel <= tol || broke) st.active[r] = 0;
  st.scale[r] = (broke || hn == 0.0) ? 0.0 : 1.0 / hn;
}

// Solve H[0:k, 0:k] y = g[0:k] (upper triangular) per right-hand side.
__global__ void backsolve_kernel(GmresState st, int R) {
  const int r = threadIdx.x;
  if (r >= R) return;
  const int m = st.m, ld = m + 1, k = st.k[r];
  for (int i = k - 1; i >= 0; --i) {
    double2 s = st.g[r * ld + i];
    for (int c = i + 1; c < k; ++c) {
      const double2 p = cmul(st.H[((int64_t)r * m + c) * ld + i], st.y[r * m + c]);
      s.x -= p.x;
      s.y -= p.y;
    }
    const double2 d = st.H[((int64_t)r * m + i) * ld + i];
    const double dd = d.x * d.x + d.y * d.y;
    st.y[r * m + i] = make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd);
  }
}

// x[r][i] += sum_{c < k[r]} V_c[r][i] y[r][c]  (FP64 sum)
__global__ __launch_bounds__(kThreads) void combine_kernel(const float2* __restrict__ V,
                                                           int64_t vstride, GmresState st,
                                                           float2* __restrict__ x, int64_t n,
                                                           int R) {
  __shared__ double2 ys[kMaxRestart];
  const int r = blockIdx.y;
  const int k = st.k[r];
  for (int c = threadIdx.x; c < k; c += kThreads) ys[c] = st.y[r * st.m + c];
  __syncthreads();
  if (k == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double2 s = f2d(x[(int64_t)r * n + i]);
    for (int c = 0; c < k; ++c) {
      const double2 p = cmul(f2d(V[(int64_t)c * vstride + (int64_t)r * n + i]), ys[c]);
      s.x += p.x;
      s.y += p.y;
    }
    x[(int64_t)r * n + i] = make_float2((float)s.x, (float)s.y);
  }
}

// Status rows for the host: res, active, iters per right-hand side.
__global__ void status_kernel(GmresState st, int R, GmresStatusRow* out) {
  const int r = threadIdx.x;
  if (r >= R) return;
  out[r].res = st.res[r];
  out[r].active = st.active[r];
  out[r].iters = st.iters[r];
}

__global__ __launch_bounds__(kThreads) void zero_kernel(float2* __restrict__ p, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads)
    p[i] = make_float2(0.f, 0.f);
}

// v[i] = (u(2i), u(2i+1)), u uniform in [-1, 1) from a 64-bit counter hash
// (the finaliser of SplitMix64) of (seed, index): a reproducible start
// vector with no host transfer.
__device__ inline double hash_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kThreads) void rand_fill_kernel(float2* __restrict__ v, int64_t n,
                                                             uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    v[i] = make_float2((float)hash_uniform(seed, 2 * i), (float)hash_uniform(seed, 2 * i + 1));
}

// dst = conj(src)
__global__ __launch_bounds__(kThreads) void conj_kernel(float2* __restrict__ dst,
                                                        const float2* __restrict__ src,
                                                        int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const float2 v = src[i];
    dst[i] = make_float2(v.x, -v.y);
  }
}

// scale[0] = 1 / sqrt(nrm[0].x)  (0 for a zero vector)
__global__ void inv_norm_kernel(const double2* __restrict__ nrm, double* __restrict__ scale) {
  if (threadIdx.x == 0) {
    const double n2 = nrm[0].x;
    scale[0] = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  }
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : (b > kDotBlocks ? kDotBlocks : b));
}

}  // namespace

int gmres_dot_blocks(int64_t n) { return (int)grid_for(n); }

int launch_gmres_dots(const float2* V, int64_t vstride, int ncol, const float2* w, int64_t n,
                      int R, double2* partial, double2* out, int ldo, hipStream_t s) {
  const unsigned nb = grid_for(n);
  const int ldp = kMaxRestart + 1;
  hipLaunchKernelGGL(dots_kernel, dim3(nb, R), dim3(kThreads), 0, s, V, vstride, ncol, w, n,
                     R, partial, ldp);
  hipLaunchKernelGGL(reduce_kernel, dim3(R), dim3(64), 0, s, partial, (int)nb, R, ncol, ldp,
                     out, ldo);
  return (int)hipGetLastError();
}

int launch_gmres_update(const float2* V, int64_t vstride, int ncol, const double2* h, int ldh,
                        float2* w, int64_t n, int R, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(grid_for(n), R), dim3(kThreads), 0, s, V, vstride,
                     ncol, h, ldh, w, n, R);
  return (int)hipGetLastError();
}

int launch_gmres_add_shift(float2* w, const float2* v, double sr, double si, int64_t total,
                           hipStream_t s) {
  hipLaunchKernelGGL(add_shift_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, w, v, sr,
                     si, total);
  return (int)hipGetLastError();
}

int launch_gmres_scale(float2* dst, const float2* src, const double* sc, int64_t n, int R,
                       hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n), R), dim3(kThreads), 0, s, dst, src, sc, n,
                     R);
  return (int)hipGetLastError();
}

int launch_gmres_residual(float2* dst, const float2* b, const float2* x, const float2* ax,
                          double sr, double si, int64_t total, hipStream_t s) {
  hipLaunchKernelGGL(residual_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, dst, b, x,
                     ax, sr, si, total);
  return (int)hipGetLastError();
}

int launch_gmres_cycle_start(const GmresState& st, int R, int first, double tol,
                             hipStream_t s) {
  hipLaunchKernelGGL(cycle_start_kernel, dim3(1), dim3(64), 0, s, st, R, first, tol);
  return (int)hipGetLastError();
}

int launch_gmres_tail(const GmresState& st, int R, int j, double tol, hipStream_t s) {
  hipLaunchKernelGGL(arnoldi_tail_kernel, dim3(1), dim3(64), 0, s, st, R, j, tol);
  return (int)hipGetLastError();
}

int launch_gmres_backsolve(const GmresState& st, int R, hipStream_t s) {
  hipLaunchKernelGGL(backsolve_kernel, dim3(1), dim3(64), 0, s, st, R);
  return (int)hipGetLastError();
}

int launch_gmres_combine(const float2* V, int64_t vstride, const GmresState& st, float2* x,
                         int64_t n, int R, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3(grid_for(n), R), dim3(kThreads), 0, s, V, vstride,
                     st, x, n, R);
  return (int)hipGetLastError();
}

int launch_gmres_status(const GmresState& st, int R, GmresStatusRow* out, hipStream_t s) {
  hipLaunchKernelGGL(status_kernel, dim3(1), dim3(64), 0, s, st, R, out);
  return (int)hipGetLastError();
}

int launch_gmres_rand(float2* v, int64_t n, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(rand_fill_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, v, n, seed);
  return (int)hipGetLastError();
}

int launch_gmres_conj(float2* dst, const float2* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(conj_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, dst, src, n);
  return (int)hipGetLastError();
}

int launch_gmres_inv_norm(const double2* nrm, double* scale, hipStream_t s) {
  hipLaunchKernelGGL(inv_norm_kernel, dim3(1), dim3(64), 0, s, nrm, scale);
  return (int)hipGetLastError();
}

int launch_gmres_zero(float2* p, int64_t total, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, p, total);
  return (int)hipGetLastError();
}

}  // namespace ubf

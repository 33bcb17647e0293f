// HIP kernels of the far-zone product for gfx950 (CDNA4).
//
// Box vectors (uniform-basis coefficients P and fields E) are kept planar
// and padded in the workspace: [re(N_u), 0.. | im(N_u), 0..], 2*kh floats
// per box (kh = N_u + 1 rounded up to even), which is also the K-axis
// layout the matrix-core translation consumes.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ubf {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup ids are dealt round-robin to the 8 XCDs (id % 8). Remap so that
// XCD x works on a contiguous block of chunks; chunks are grouped by offset,
// so each XCD's L2 only holds the operators of its own offsets. `grid` is a
// multiple of 8.
__device__ inline int xcd_chunk(int bid, int grid) {
  const int per = grid >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// ---------------------------------------------------------------- layout

__global__ __launch_bounds__(kBlock) void pack_kernel(
    const float2* __restrict__ x, float* __restrict__ P, int64_t n_rows,
    int nu, int kh) {
  const int64_t total = n_rows * kh;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(t % kh);
    const int64_t row = t / kh;
    const float2 v = u < nu ? x[row * nu + u] : make_float2(0.f, 0.f);
    P[row * 2 * kh + u] = v.x;
    P[row * 2 * kh + kh + u] = v.y;
  }
}

__global__ __launch_bounds__(kBlock) void unpack_kernel(
    const float* __restrict__ P, float2* __restrict__ out, int64_t n_rows,
    int nu, int kh) {
  const int64_t total = n_rows * nu;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(t % nu);
    const int64_t row = t / nu;
    out[t] = make_float2(P[row * 2 * kh + u], P[row * 2 * kh + kh + u]);
  }
}

// ---------------------------------------------------------------- stage 1

// One workgroup per (box, rhs). Thread t owns row u = t % nu of S_i and
// column group g = t / nu, so thread t reads S_i element t + nu*G*it: the
// whole block streams S_i contiguously. The G column-group partial sums
// are reduced through LDS.
__global__ __launch_bounds__(kBlock) void aggregate_kernel(
    const float2* __restrict__ x, const int64_t* __restrict__ nb_ptr,
    const float2* __restrict__ S, float* __restrict__ P, int64_t n_box,
    int64_t nb_total, int nu, int kh) {
  __shared__ float2 red[kBlock];
  const int64_t i = blockIdx.x;
  const int r = blockIdx.y;
  const int t = threadIdx.x;
  const int G = kBlock / nu;
  const int u = t % nu, g = t / nu;
  const int64_t start = nb_ptr[i];
  const int64_t nb = nb_ptr[i + 1] - start;
  const float2* Sb = S + start * nu;
  const float2* xb = x + (int64_t)r * nb_total + start;
  float ar = 0.f, ai = 0.f;
  if (g < G) {
    for (int64_t c = g; c < nb; c += G) {
      const float2 s = Sb[c * nu + u];
      const float2 xv = xb[c];
      ar = fmaf(s.x, xv.x, ar);
      ar = fmaf(-s.y, xv.y, ar);
      ai = fmaf(s.x, xv.y, ai);
      ai = fmaf(s.y, xv.x, ai);
    }
  }
  red[t] = make_float2(ar, ai);
  __syncthreads();
  float* Pb = P + ((int64_t)r * n_box + i) * 2 * kh;
  for (int v = t; v < kh; v += kBlock) {
    float sr = 0.f, si = 0.f;
    if (v < nu)
      for (int gg = 0; gg < G; ++gg) {
        sr += red[gg * nu + v].x;
        si += red[gg * nu + v].y;
      }
    Pb[v] = sr;
    Pb[kh + v] = si;
  }
}

// ---------------------------------------------------------------- stage 2

// Matrix-core translation, one workgroup per (chunk, rhs): a chunk is up to
// 64 box pairs sharing one offset w. The complex product E = G_w P is done
// as the real product
//   [Er; Ei] = [[Gr, -Gi], [Gi, Gr]] [Pr; Pi]
// with M = 2*NU output rows (padded to 16-row blocks) and K = 2*KH.
// G_w is staged in LDS as its two planes; each wavefront owns 16 pair
// columns, holds their K values in registers, and sweeps all row blocks
// with v_mfma_f32_16x16x4_f32. The K axis is split into four quadrants of
// QK values, one per 16-lane group, so each lane loads a contiguous run of
// its column and the operator read for a k-step is an immediate offset.
template <int NU>
__global__ __launch_bounds__(kBlock, 2) void translate_mfma_kernel(
    const float* __restrict__ table, const int32_t* __restrict__ chunks,
    int n_chunks, const int32_t* __restrict__ pair_src,
    const float* __restrict__ P, float* __restrict__ part, int64_t n_box,
    int64_t n_pairs) {
  constexpr int KH = (NU + 2) & ~1;
  constexpr int QK = KH / 2;
  constexpr int PLANE = (NU + 1) * KH;
  constexpr int M = 2 * NU;
  constexpr int RB = (M + 15) / 16;
  constexpr int PSTR = 2 * KH;
  __shared__ float lds[2 * PLANE];

  const int chunk = xcd_chunk(blockIdx.x, gridDim.x);
  if (chunk >= n_chunks) return;
  const int rhs = blockIdx.y;
  const int o = chunks[4 * chunk];
  const int begin = chunks[4 * chunk + 1];
  const int count = chunks[4 * chunk + 2];

  const float4* g4 = reinterpret_cast<const float4*>(table + (size_t)o * 2 * PLANE);
  float4* l4 = reinterpret_cast<float4*>(lds);
  for (int i = threadIdx.x; i < 2 * PLANE / 4; i += kBlock) l4[i] = g4[i];
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col0 = wave * 16;
  if (col0 >= count) return;  // no barrier follows
  const int n = lane & 15, q = lane >> 4;
  const int c = col0 + n;
  const bool valid = c < count;
  const int64_t pos = (int64_t)begin + c;
  const int src = valid ? pair_src[pos] : 0;
  const float* pb = P + ((int64_t)rhs * n_box + src) * PSTR + q * QK;

  float b[QK];
#pragma unroll
  for (int ks = 0; ks < QK; ++ks) b[ks] = valid ? pb[ks] : 0.f;

  const bool khalf_im = q >= 2;
  const int colb = (q & 1) * QK;
  int base[RB];
  unsigned sgn[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int row = rb * 16 + n;
    const bool in_rows = row < M;
    const bool out_im = row >= NU;
    const int rr = in_rows ? (out_im ? row - NU : row) : NU;  // NU: zero row
    const int plane = (khalf_im != out_im) ? 1 : 0;
    base[rb] = plane * PLANE + rr * KH + colb;
    sgn[rb] = (khalf_im && !out_im) ? 0x80000000u : 0u;
  }

  floatx4 acc[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int ks = 0; ks < QK; ++ks) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const float a = __uint_as_float(__float_as_uint(lds[base[rb] + ks]) ^ sgn[rb]);
      acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks], acc[rb], 0, 0, 0);
    }
  }

  if (valid) {
    float* out = part + ((int64_t)rhs * n_pairs + pos) * PSTR;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int r0 = rb * 16 + q * 4;
      if (r0 < PSTR) *reinterpret_cast<floatx4*>(out + r0) = acc[rb];
    }
  }
}

// Plain translation for box sizes without a matrix-core variant: one
// workgroup per (chunk, rhs), one thread per output row, operator rows read
// from the table through the cache.
__global__ __launch_bounds__(kBlock) void translate_generic_kernel(
    const float* __restrict__ table, const int32_t* __restrict__ chunks,
    const int32_t* __restrict__ pair_src, const float* __restrict__ P,
    float* __restrict__ part, int64_t n_box, int64_t n_pairs, int nu, int kh) {
  __shared__ float pv[2 * 196];
  const int chunk = blockIdx.x;
  const int rhs = blockIdx.y;
  const int o = chunks[4 * chunk];
  const int begin = chunks[4 * chunk + 1];
  const int count = chunks[4 * chunk + 2];
  const size_t plane = (size_t)(nu + 1) * kh;
  const float* Gr = table + (size_t)o * 2 * plane;
  const float* Gi = Gr + plane;
  const int pstr = 2 * kh;
  for (int c = 0; c < count; ++c) {
    const int64_t pos = (int64_t)begin + c;
    const int src = pair_src[pos];
    __syncthreads();
    for (int t = threadIdx.x; t < pstr; t += kBlock)
      pv[t] = P[((int64_t)rhs * n_box + src) * pstr + t];
    __syncthreads();
    for (int m = threadIdx.x; m < 2 * nu; m += kBlock) {
      const bool im = m >= nu;
      const int rr = im ? m - nu : m;
      const float* gr = Gr + (size_t)rr * kh;
      const float* gi = Gi + (size_t)rr * kh;
      float s = 0.f;
      if (im) {
        for (int v = 0; v < nu; ++v) s = fmaf(gi[v], pv[v], fmaf(gr[v], pv[kh + v], s));
      } else {
        for (int v = 0; v < nu; ++v) s = fmaf(gr[v], pv[v], fmaf(-gi[v], pv[kh + v], s));
      }
      part[((int64_t)rhs * n_pairs + pos) * pstr + m] = s;
    }
  }
}

// ---------------------------------------------------------------- stage 3

// One workgroup per (test box, rhs). E_j is first gathered into LDS, either
// as the sum of the box's partial products or from a complex input vector.
// mode 0: identity basis (y_j = E_j); mode 1: T_j = S_j^T, one wavefront
// per column of S_j with a wave reduction; mode 2: explicit column-major
// T_j, one thread per output row.
template <bool FROM_PARTS>
__global__ __launch_bounds__(kBlock) void disaggregate_kernel(
    const float* __restrict__ part, const int32_t* __restrict__ test_ptr,
    const int32_t* __restrict__ test_pos, int64_t n_pairs,
    const float2* __restrict__ Ein, const int64_t* __restrict__ nb_ptr,
    const float2* __restrict__ S, const float2* __restrict__ T, int mode,
    float2* __restrict__ y, int64_t n_box, int64_t nb_total, int nu, int kh) {
  __shared__ float Es[2 * 192];
  const int64_t j = blockIdx.x;
  const int r = blockIdx.y;
  const int t = threadIdx.x;
  if (FROM_PARTS) {
    const int p0 = test_ptr[j], p1 = test_ptr[j + 1];
    const float* pr = part + (int64_t)r * n_pairs * 2 * kh;
    for (int m = t; m < 2 * nu; m += kBlock) {
      float s = 0.f;
      for (int p = p0; p < p1; ++p) s += pr[(int64_t)test_pos[p] * 2 * kh + m];
      Es[m] = s;
    }
  } else {
    for (int u = t; u < nu; u += kBlock) {
      const float2 e = Ein[((int64_t)r * n_box + j) * nu + u];
      Es[u] = e.x;
      Es[nu + u] = e.y;
    }
  }
  __syncthreads();
  float2* yb = y + (int64_t)r * nb_total;
  if (mode == 0) {
    for (int u = t; u < nu; u += kBlock) yb[j * nu + u] = make_float2(Es[u], Es[nu + u]);
    return;
  }
  const int64_t start = nb_ptr[j];
  const int64_t nb = nb_ptr[j + 1] - start;
  if (mode == 1) {
    const int wave = t >> 6, lane = t & 63;
    for (int64_t c = wave; c < nb; c += kBlock / 64) {
      const float2* col = S + (start + c) * nu;
      float sr = 0.f, si = 0.f;
      for (int u = lane; u < nu; u += 64) {
        const float2 s = col[u];
        const float er = Es[u], ei = Es[nu + u];
        sr = fmaf(s.x, er, fmaf(-s.y, ei, sr));
        si = fmaf(s.x, ei, fmaf(s.y, er, si));
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      if (lane == 0) yb[start + c] = make_float2(sr, si);
    }
  } else {
    const float2* Tb = T + start * nu;
    for (int64_t c = t; c < nb; c += kBlock) {
      float sr = 0.f, si = 0.f;
      for (int u = 0; u < nu; ++u) {
        const float2 v = Tb[c + nb * u];
        const float er = Es[u], ei = Es[nu + u];
        sr = fmaf(v.x, er, fmaf(-v.y, ei, sr));
        si = fmaf(v.x, ei, fmaf(v.y, er, si));
      }
      yb[start + c] = make_float2(sr, si);
    }
  }
}

int grid_for(int64_t total) {
  const int64_t g = (total + kBlock - 1) / kBlock;
  return (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

}  // namespace

bool translate_uses_mfma(const Plan& p) {
  return p.nu == 81 || p.nu == 24 || p.nu == 3;
}

int launch_pack(const Plan& p, const void* x, float* P, int nrhs, void* stream) {
  const int64_t rows = (int64_t)nrhs * p.n_box;
  hipLaunchKernelGGL(pack_kernel, dim3(grid_for(rows * p.kh)), dim3(kBlock), 0,
                     (hipStream_t)stream, (const float2*)x, P, rows, p.nu, p.kh);
  return (int)hipGetLastError();
}

int launch_unpack(const Plan& p, const float* P, void* out, int nrhs, void* stream) {
  const int64_t rows = (int64_t)nrhs * p.n_box;
  hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(rows * p.nu)), dim3(kBlock), 0,
                     (hipStream_t)stream, P, (float2*)out, rows, p.nu, p.kh);
  return (int)hipGetLastError();
}

int launch_aggregate(const Plan& p, const void* x, float* P, int nrhs, void* stream) {
  if (!p.has_basis) return launch_pack(p, x, P, nrhs, stream);
  hipLaunchKernelGGL(aggregate_kernel, dim3((unsigned)p.n_box, nrhs), dim3(kBlock), 0,
                     (hipStream_t)stream, (const float2*)x, p.d_nb_ptr,
                     (const float2*)p.d_S, P, p.n_box, p.nb_total(), p.nu, p.kh);
  return (int)hipGetLastError();
}

int launch_translate(const Plan& p, const float* P, float* part, int nrhs,
                     void* stream) {
  const int nch = (int)p.n_chunks();
  if (nch == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid8((unsigned)((nch + 7) / 8 * 8), nrhs);
  switch (p.nu) {
    case 81:
      hipLaunchKernelGGL(translate_mfma_kernel<81>, grid8, dim3(kBlock), 0, s,
                         p.d_table, p.d_chunks, nch, p.d_pair_src, P, part,
                         p.n_box, p.n_pairs());
      break;
    case 24:
      hipLaunchKernelGGL(translate_mfma_kernel<24>, grid8, dim3(kBlock), 0, s,
                         p.d_table, p.d_chunks, nch, p.d_pair_src, P, part,
                         p.n_box, p.n_pairs());
      break;
    case 3:
      hipLaunchKernelGGL(translate_mfma_kernel<3>, grid8, dim3(kBlock), 0, s,
                         p.d_table, p.d_chunks, nch, p.d_pair_src, P, part,
                         p.n_box, p.n_pairs());
      break;
    default:
      hipLaunchKernelGGL(translate_generic_kernel, dim3((unsigned)nch, nrhs),
                         dim3(kBlock), 0, s, p.d_table, p.d_chunks, p.d_pair_src,
                         P, part, p.n_box, p.n_pairs(), p.nu, p.kh);
  }
  return (int)hipGetLastError();
}

int launch_disaggregate(const Plan& p, bool from_parts, const float* part,
                        const void* E, void* y, int nrhs, void* stream,
                        bool identity) {
  const int mode = (identity || !p.has_basis) ? 0 : (p.d_T ? 2 : 1);
  const int64_t nb_total = mode == 0 ? p.n_box * (int64_t)p.nu : p.nb_total();
  const dim3 grid((unsigned)p.n_box, nrhs);
  hipStream_t s = (hipStream_t)stream;
  if (from_parts)
    hipLaunchKernelGGL(disaggregate_kernel<true>, grid, dim3(kBlock), 0, s, part,
                       p.d_test_ptr, p.d_test_pos, p.n_pairs(), (const float2*)E,
                       p.d_nb_ptr, (const float2*)p.d_S, (const float2*)p.d_T, mode,
                       (float2*)y, p.n_box, nb_total, p.nu, p.kh);
  else
    hipLaunchKernelGGL(disaggregate_kernel<false>, grid, dim3(kBlock), 0, s, part,
                       p.d_test_ptr, p.d_test_pos, p.n_pairs(), (const float2*)E,
                       p.d_nb_ptr, (const float2*)p.d_S, (const float2*)p.d_T, mode,
                       (float2*)y, p.n_box, nb_total, p.nu, p.kh);
  return (int)hipGetLastError();
}

}  // namespace ubf

// HIP kernels of the far-zone product for gfx950 (CDNA4).
//
// Box vectors (uniform-basis coefficients P and fields E) are kept planar
// and padded in the workspace: [re(N_u), 0.. | im(N_u), 0..], 2*kh floats
// per box (kh = N_u + 1 rounded up to even), which is also the K-axis
// layout the matrix-core translation consumes.
#include <algorithm>

#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ubf {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned uintx4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs), and back.
__device__ inline unsigned bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf16_f(unsigned b) { return __uint_as_float(b << 16); }

// Round-to-nearest FP32 -> FP16 bits, and back.
__device__ inline unsigned short f16_rn(float f) { return __half_as_ushort(__float2half_rn(f)); }
__device__ inline float f16_f(unsigned short b) { return __half2float(__ushort_as_half(b)); }

// Index of part `part` (0 re.hi, 1 im.hi, 2 re.lo, 3 im.lo) of coefficient
// u in a 16-bit box vector: groups of 8 coefficients (one matrix-core
// k-step) interleave the four parts, [re.hi(8) im.hi(8) re.lo(8) im.lo(8)],
// so the two lanes holding a column's K halves read adjacent 16 bytes.
__device__ inline int q16(int part, int u) { return 32 * (u >> 3) + 8 * part + (u & 7); }

// Writes one box-vector coefficient (re, im) at index u of a box vector
// starting at Pb. mode 0: FP32 layout [re(kh) | im(kh)]. Otherwise the
// 16-bit layout of q16 (khb coefficients), with hi = round(v),
// lo = round(v - hi): mode 1 in BF16; mode 2 in FP16 of v * inv_scale (the
// box vector's power-of-two scale).
__device__ inline void put_coef(float* Pb, int u, float re, float im, int kh, int khb,
                                int mode, float inv_scale = 1.f) {
  if (mode == 0) {
    Pb[u] = re;
    Pb[kh + u] = im;
    return;
  }
  unsigned short* q = reinterpret_cast<unsigned short*>(Pb);
  if (mode == 1) {
    const unsigned rh = bf16_rne(re), ih = bf16_rne(im);
    q[q16(0, u)] = (unsigned short)rh;
    q[q16(2, u)] = (unsigned short)bf16_rne(re - bf16_f(rh));
    q[q16(1, u)] = (unsigned short)ih;
    q[q16(3, u)] = (unsigned short)bf16_rne(im - bf16_f(ih));
    return;
  }
  re *= inv_scale;  // exact: a power of two
  im *= inv_scale;
  const unsigned short rh = f16_rn(re), ih = f16_rn(im);
  q[q16(0, u)] = rh;
  q[q16(2, u)] = f16_rn(re - f16_f(rh));
  q[q16(1, u)] = ih;
  q[q16(3, u)] = f16_rn(im - f16_f(ih));
}

// Power-of-two scale bringing a box vector's largest |Re|, |Im| to
// [2^14, 2^15) (1 for a zero vector). The exponent is held at -126 or
// above, so the scale is a normal float and its inverse (at most 2^126) is
// finite and exact; a vector whose largest part is below 2^-112 is then
// scaled up by 2^126 only, which still leaves that part within FP16 range.
__device__ inline float box_scale_for(float maxabs) {
  if (!(maxabs > 0.f)) return 1.f;
  return ldexpf(1.f, max(ilogbf(maxabs) - 14, -126));
}

constexpr int kBlock = 256;

// A partial row is read once, by stage 3 of the same product: load it
// without keeping it in the caches, which leaves their room to the data the
// next stages reuse (the operator table and the basis; measured: stage 2
// of the next product 38.5 -> 33.6 us on the 3,338-box shell).
__device__ inline float4 load_once(const float4* p) {
  const floatx4 q = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(p));
  return make_float4(q.x, q.y, q.z, q.w);
}


// Workgroup ids are dealt round-robin to the 8 XCDs (id % 8). Remap so that
// XCD x works on a contiguous block of work; work is grouped by offset, so
// each XCD's L2 only holds the operators of its own offsets. `grid` is a
// multiple of 8.
__device__ inline int xcd_chunk(int bid, int grid) {
  const int per = grid >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Partial rows of one 32x32 accumulator block (32 columns of a wavefront,
// rows m0..m0+31 of each column's partial row) are written through a
// per-wavefront LDS tile: the block's D layout gives a lane 4-row pieces of
// one column, so direct stores touch 32 rows per instruction; after the
// transpose, lane l stores 16 bytes of column (l / 8) + 8 * it, and one
// store instruction covers 8 columns x 128 contiguous bytes. Columns'
// destination rows (within the RHS's block `part_rhs`) are taken from their
// owning lanes; absent columns (c >= ncol) and rows at or past `pstr` are
// not stored (masked stores). The tile pitch of 36 floats keeps the
// 16-byte writes conflict-free. LDS accesses of one wavefront execute in
// order, so the tile needs no barrier.
constexpr int kTilePitch = 36;
__device__ inline void store_block_transposed(float* tile, const floatx16& acc, float sc,
                                              int dst, int ncol, float* __restrict__ part_rhs,
                                              int pstr, int m0) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4)
    *reinterpret_cast<floatx4*>(tile + r * kTilePitch + 8 * q4 + 4 * h) =
        floatx4{acc[4 * q4], acc[4 * q4 + 1], acc[4 * q4 + 2], acc[4 * q4 + 3]} * sc;
  const int seg = lane & 7;
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int c = (lane >> 3) + 8 * it;
    const floatx4 v = *reinterpret_cast<const floatx4*>(tile + c * kTilePitch + 4 * seg);
    const int m = m0 + 4 * seg;
    const int row = __shfl(dst, c, 64);  // column c's destination row
    if (c < ncol && m + 4 <= pstr)
      *reinterpret_cast<floatx4*>(part_rhs + (int64_t)row * pstr + m) = v;
  }
}

// ---------------------------------------------------------------- layout

__global__ __launch_bounds__(kBlock) void pack_kernel(
    const float2* __restrict__ x, float* __restrict__ P, int64_t n_rows,
    int nu, int kh, int khb, int mode) {
  const int len = mode ? khb : kh;             // coefficients incl. zero pad
  const int vs = mode ? 2 * khb : 2 * kh;      // box vector stride (floats)
  const int64_t total = n_rows * len;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(t % len);
    const int64_t row = t / len;
    const float2 v = u < nu ? x[row * nu + u] : make_float2(0.f, 0.f);
    put_coef(P + row * vs, u, v.x, v.y, kh, khb, mode);
  }
}

// FP16 forms: one wavefront per box vector (row), four per workgroup; the
// vector's scale needs its largest component first. nu <= 192 (three
// coefficients per lane).
__global__ __launch_bounds__(kBlock) void pack_f16_kernel(
    const float2* __restrict__ x, float* __restrict__ P, float* __restrict__ box_scale,
    int nu, int khb, int64_t n_rows) {
  const int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (row >= n_rows) return;  // whole wavefronts
  const int l = threadIdx.x & 63;
  float2 v[3];
  float m = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int u = l + 64 * i;
    v[i] = u < nu ? x[row * nu + u] : make_float2(0.f, 0.f);
    m = fmaxf(m, fmaxf(fabsf(v[i].x), fabsf(v[i].y)));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  const float sc = box_scale_for(m);
  const float inv = 1.f / sc;
  float* Pb = P + row * 2 * khb;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (l + 64 * i < khb) put_coef(Pb, l + 64 * i, v[i].x, v[i].y, 0, khb, 2, inv);
  if (l == 0) box_scale[row] = sc;
}

__global__ __launch_bounds__(kBlock) void unpack_kernel(
    const float* __restrict__ P, float2* __restrict__ out, int64_t n_rows,
    int nu, int kh, int khb, int mode, const float* __restrict__ box_scale) {
  const int vs = mode ? 2 * khb : 2 * kh;
  const int64_t total = n_rows * nu;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(t % nu);
    const int64_t row = t / nu;
    const float* Pb = P + row * vs;
    const unsigned short* q = reinterpret_cast<const unsigned short*>(Pb);
    if (mode == 0) {
      out[t] = make_float2(Pb[u], Pb[kh + u]);
    } else if (mode == 1) {
      out[t] = make_float2(bf16_f(q[q16(0, u)]) + bf16_f(q[q16(2, u)]),
                           bf16_f(q[q16(1, u)]) + bf16_f(q[q16(3, u)]));
    } else {
      const float sc = box_scale[row];
      out[t] = make_float2((f16_f(q[q16(0, u)]) + f16_f(q[q16(2, u)])) * sc,
                           (f16_f(q[q16(1, u)]) + f16_f(q[q16(3, u)])) * sc);
    }
  }
}

// ---------------------------------------------------------------- stage 1

// One workgroup per (box, block of RB right-hand sides). Thread t owns row
// u = t % nu of S_i and column group g = t / nu, so thread t reads S_i
// element t + nu*G*it: the whole block streams S_i contiguously, once for
// the RB vectors. The G column-group partial sums are reduced through LDS.
template <int RB>
__global__ __launch_bounds__(kBlock) void aggregate_kernel(
    const float2* __restrict__ x, const int64_t* __restrict__ nb_ptr,
    const float2* __restrict__ S, float* __restrict__ P, int64_t n_box,
    int64_t nb_total, int nu, int kh, int khb, int mode, float* __restrict__ box_scale,
    int nrhs) {
  __shared__ float2 red[RB][kBlock];
  __shared__ float wmax[kBlock / 64];
  const int64_t i = blockIdx.x;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);  // >= 1
  const int t = threadIdx.x;
  const int G = kBlock / nu;
  const int u = t % nu, g = t / nu;
  const int64_t start = nb_ptr[i];
  const int64_t nb = nb_ptr[i + 1] - start;
  const float2* Sb = S + start * nu;
  const float2* xb = x + (int64_t)r0 * nb_total + start;
  float ar[RB], ai[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) ar[q] = ai[q] = 0.f;
  if constexpr (RB == 1) {
    if (g < G) {
#pragma unroll 9
      for (int64_t c = g; c < nb; c += G) {
        const float2 s = Sb[c * nu + u];
        const float2 xv = xb[c];
        ar[0] = fmaf(s.x, xv.x, ar[0]);
        ar[0] = fmaf(-s.y, xv.y, ar[0]);
        ai[0] = fmaf(s.x, xv.y, ai[0]);
        ai[0] = fmaf(s.y, xv.x, ai[0]);
      }
    }
  } else {
    // the block's x values go through LDS, 256 columns at a time, so that
    // the loop's only global loads are those of S_i; vectors past the last
    // one repeat it, and their sums are not stored
    __shared__ float2 xs[RB][kBlock];
    for (int64_t c0 = 0; c0 < nb; c0 += kBlock) {
      const int64_t cn = min<int64_t>(kBlock, nb - c0);
      if (c0 > 0) __syncthreads();  // every thread is done with the last tile
#pragma unroll
      for (int q = 0; q < RB; ++q)
        if (t < cn) xs[q][t] = xb[(int64_t)min(q, nr - 1) * nb_total + c0 + t];
      __syncthreads();
      if (g < G) {
#pragma unroll 5
        for (int c = g; c < cn; c += G) {
          const float2 s = Sb[(c0 + c) * nu + u];
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            const float2 xv = xs[q][c];
            ar[q] = fmaf(s.x, xv.x, ar[q]);
            ar[q] = fmaf(-s.y, xv.y, ar[q]);
            ai[q] = fmaf(s.x, xv.y, ai[q]);
            ai[q] = fmaf(s.y, xv.x, ai[q]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RB; ++q) red[q][t] = make_float2(ar[q], ai[q]);
  __syncthreads();
  const int len = mode ? khb : kh;  // <= kBlock: one coefficient per thread
  for (int q = 0; q < nr; ++q) {
    const int r = r0 + q;
    float* Pb = P + ((int64_t)r * n_box + i) * (mode ? 2 * khb : 2 * kh);
    float sr = 0.f, si = 0.f;
    if (t < nu)
      for (int gg = 0; gg < G; ++gg) {
        sr += red[q][gg * nu + t].x;
        si += red[q][gg * nu + t].y;
      }
    float inv = 1.f;
    if (mode == 2) {  // FP16: the box vector's scale from its largest component
      float m = fmaxf(fabsf(sr), fabsf(si));
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
      if ((t & 63) == 0) wmax[t >> 6] = m;
      __syncthreads();
      m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
      if (q + 1 < nr) __syncthreads();  // wmax is reused by the next vector
      const float sc = box_scale_for(m);
      inv = 1.f / sc;
      if (t == 0) box_scale[(int64_t)r * n_box + i] = sc;
    }
    if (t < len) put_coef(Pb, t, sr, si, kh, khb, mode, inv);
  }
}

// ---------------------------------------------------------------- stage 2

// Waits until at most N vector-memory operations of this wavefront are
// outstanding (vmcnt; expcnt and lgkmcnt left unconstrained).
template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Workgroup barrier once every wavefront's LDS reads have returned (so LDS
// may be overwritten afterwards). Unlike __syncthreads it does not wait for
// outstanding global loads and stores.
__device__ inline void lds_reads_done_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroup barrier after each wavefront has waited for its own direct
// copies into LDS (wait_vmcnt): LDS reads after it see every wavefront's
// copied data.
__device__ inline void lds_copies_done_barrier() {
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Direct copy of N16 16-byte units from global memory into LDS (no
// registers): round `it` of the workgroup copies units it*kBlock + t, and
// wavefront w's 64 lanes fill the 1 KB at dst + it*kBlock + 64 w (the
// copy's LDS address is the wavefront's base plus 16 bytes per lane). `dst`
// holds ceil(N16 / kBlock) * kBlock units; lanes past N16 read the last
// unit into padding. Issues ceil(N16 / kBlock) loads per thread.
template <int N16>
__device__ inline void copy_to_lds(const uintx4* __restrict__ src, uintx4* dst) {
  const int t = threadIdx.x, wave = t >> 6;
#pragma unroll
  for (int it = 0; it < (N16 + kBlock - 1) / kBlock; ++it)
    __builtin_amdgcn_global_load_lds(
        reinterpret_cast<const void*>(src + min(t + it * kBlock, N16 - 1)),
        (__attribute__((address_space(3))) void*)(dst + it * kBlock + wave * 64), 16, 0, 0);
}

// Matrix-core translation. A chunk is up to 128 box pairs sharing one
// offset w; each workgroup walks a contiguous range of chunks (grouped by
// offset, so consecutive chunks mostly reuse the operator already staged).
// The complex product E = G_w P is done as the real product
//   [Er; Ei] = [[Gr, -Gi], [Gi, Gr]] [Pr; Pi]
// on v_mfma_f32_32x32x2_f32: M = 2*NU output rows in 32-row blocks,
// K = 2*NU. Each wavefront owns 32 pair columns. Lane l holds column
// l % 32 and K half h = l / 32 (h = 0: the Pr terms, h = 1: the Pi terms),
// so a k-step of the MFMA pairs k = ks (h = 0) with k = NU + ks (h = 1) and
// each lane's B values are one contiguous run of its box vector, kept in
// registers. G_w sits in LDS as its two planes (rows of PITCH floats);
// a lane reads the A values of four consecutive k-steps with one 16-byte
// LDS read, negating -Gi with a sign flip. Operators are copied global ->
// LDS directly: the first before the loop, each later one (when the next
// chunk has another offset) after every wavefront's last products and
// before the partial rows leave, so that the copy is in flight with the
// stores; the next chunk then waits for both.
template <int NU>
__global__ __launch_bounds__(kBlock, 2) void translate_mfma_kernel(
    const float* __restrict__ table, const int32_t* __restrict__ chunks,
    const int32_t* __restrict__ wg_ptr, const int32_t* __restrict__ pair_src,
    const int32_t* __restrict__ pair_dst, const float* __restrict__ P,
    float* __restrict__ part, int64_t n_box, int64_t n_pairs, int64_t trash_row) {
  constexpr int KH = (NU + 3) & ~3;      // padded half-length, = PITCH
  constexpr int PLANE = NU * KH;
  constexpr int M = 2 * NU;
  // Full 32-row blocks run on the matrix cores; up to 4 leftover rows (2 for
  // N_u = 81: rows 160, 161) are accumulated on the VALU instead of a
  // mostly empty extra block. Larger remainders take a padded block.
  constexpr int LRV = (M % 32 <= 4) ? M % 32 : 0;   // VALU rows
  constexpr int RB = (M - LRV + 31) / 32;            // MFMA row blocks
  constexpr int NG = NU / 4;             // full groups of 4 k-steps
  constexpr int PSTR = 2 * KH;
  constexpr int N4 = 2 * PLANE / 4;      // 16-byte units per operator
  constexpr int HP = (N4 + kBlock - 1) / kBlock * kBlock;  // LDS units
  constexpr int NB4 = NU / 4;            // float4 loads of a lane's B run
  __shared__ uintx4 lds4[HP];
  const float* lds = reinterpret_cast<const float*>(lds4);

  const int group = xcd_chunk(blockIdx.x, gridDim.x);
  const int cbeg = wg_ptr[group], cend = wg_ptr[group + 1];
  const int rhs = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;

  // Operator addressing: output row `row` of block rb for this lane.
  // Er rows (< NU) read Gr for h = 0 and -Gi for h = 1; Ei rows read Gi for
  // h = 0 and Gr for h = 1; padding rows (>= M) read row 0 (discarded).
  int abase[RB + LRV];
  unsigned asgn[RB + LRV];
#pragma unroll
  for (int rb = 0; rb < RB + LRV; ++rb) {
    // MFMA blocks: this lane's row of block rb; VALU rows: row 32*RB + i.
    const int row = rb < RB ? rb * 32 + r : 32 * RB + (rb - RB);
    const bool er = row < NU;
    const int rr = er ? row : (row < M ? row - NU : 0);
    const bool im_plane = er ? (h == 1) : (row < M && h == 0);
    abase[rb] = (im_plane ? PLANE : 0) + rr * KH;
    asgn[rb] = (er && h == 1) ? 0x80000000u : 0u;
  }

  if (cbeg >= cend) return;
  const int col0 = wave * 32;
  const int64_t last = n_pairs - 1;

  // Every global access below is unconditional, so the in-order counter of
  // outstanding vector memory operations stays exact and waits are only as
  // deep as needed: a lane past its chunk's count reads the column of a
  // clamped (valid) pair and stores into the spare row `trash_row`; a B
  // column only feeds its own output column, so nothing else is affected.
  // Pair indices are fetched two chunks ahead (before the stores that lie
  // between), B values one chunk ahead: while k-group g of the current
  // chunk is multiplied, b's group g is refilled for the next chunk.
  int o0 = chunks[4 * cbeg], b0 = chunks[4 * cbeg + 1], n0 = chunks[4 * cbeg + 2];
  const bool has1 = cbeg + 1 < cend;
  int o1 = has1 ? chunks[4 * (cbeg + 1)] : o0;
  int b1 = has1 ? chunks[4 * (cbeg + 1) + 1] : 0;
  int n1 = has1 ? chunks[4 * (cbeg + 1) + 2] : 0;
  int64_t i0 = min((int64_t)b0 + col0 + r, last), i1 = min((int64_t)b1 + col0 + r, last);
  int src0 = pair_src[i0], dst0 = pair_dst[i0];
  int src1 = pair_src[i1], dst1 = pair_dst[i1];

  float b[NU];
  {
    const float* pb = P + ((int64_t)rhs * n_box + src0) * PSTR + h * KH;
#pragma unroll
    for (int i = 0; i < NB4; ++i) {
      const floatx4 v = reinterpret_cast<const floatx4*>(pb)[i];
      b[4 * i] = v[0];
      b[4 * i + 1] = v[1];
      b[4 * i + 2] = v[2];
      b[4 * i + 3] = v[3];
    }
#pragma unroll
    for (int ks = 4 * NB4; ks < NU; ++ks) b[ks] = pb[ks];
  }

  const uintx4* gt = reinterpret_cast<const uintx4*>(table);
  copy_to_lds<N4>(gt + (size_t)o0 * N4, lds4);
  wait_vmcnt<0>();
  lds_copies_done_barrier();
  bool pending = false;
  for (int ch = cbeg; ch < cend; ++ch) {
    if (pending) {  // uniform: the copy issued during the previous chunk
      wait_vmcnt<0>();
      lds_copies_done_barrier();
      pending = false;
    }
    const bool has2 = ch + 2 < cend;
    const int o2 = has2 ? chunks[4 * (ch + 2)] : o1;
    const int b2 = has2 ? chunks[4 * (ch + 2) + 1] : 0;
    const int n2 = has2 ? chunks[4 * (ch + 2) + 2] : 0;
    const int64_t i2 = min((int64_t)b2 + col0 + r, last);
    const float* pb1 = P + ((int64_t)rhs * n_box + src1) * PSTR + h * KH;
    int src2, dst2;

    const bool active = col0 < n0;  // wave-uniform
    floatx16 acc[RB];
    float vacc[LRV > 0 ? LRV : 1];
    if (active) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[rb] = floatx16{};
#pragma unroll
      for (int i = 0; i < LRV; ++i) vacc[i] = 0.f;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        float4 a[RB + LRV];
#pragma unroll
        for (int rb = 0; rb < RB + LRV; ++rb) {
          const float4 v = *reinterpret_cast<const float4*>(lds + abase[rb] + 4 * g);
          a[rb] = make_float4(__uint_as_float(__float_as_uint(v.x) ^ asgn[rb]),
                              __uint_as_float(__float_as_uint(v.y) ^ asgn[rb]),
                              __uint_as_float(__float_as_uint(v.z) ^ asgn[rb]),
                              __uint_as_float(__float_as_uint(v.w) ^ asgn[rb]));
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rb][jj], b[4 * g + jj], acc[rb], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < LRV; ++i) {
          vacc[i] = fmaf(a[RB + i].x, b[4 * g], vacc[i]);
          vacc[i] = fmaf(a[RB + i].y, b[4 * g + 1], vacc[i]);
          vacc[i] = fmaf(a[RB + i].z, b[4 * g + 2], vacc[i]);
          vacc[i] = fmaf(a[RB + i].w, b[4 * g + 3], vacc[i]);
        }
        const floatx4 v = reinterpret_cast<const floatx4*>(pb1)[g];  // next chunk
        b[4 * g] = v[0];
        b[4 * g + 1] = v[1];
        b[4 * g + 2] = v[2];
        b[4 * g + 3] = v[3];
      }
#pragma unroll
      for (int ks = 4 * NG; ks < NU; ++ks) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const float av = __uint_as_float(__float_as_uint(lds[abase[rb] + ks]) ^ asgn[rb]);
          acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b[ks], acc[rb], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < LRV; ++i) {
          const float av = __uint_as_float(__float_as_uint(lds[abase[RB + i] + ks]) ^ asgn[RB + i]);
          vacc[i] = fmaf(av, b[ks], vacc[i]);
        }
        b[ks] = pb1[ks];
      }
      // VALU rows: add the other K half (lane l +- 32 holds it).
#pragma unroll
      for (int i = 0; i < LRV; ++i) vacc[i] += __shfl_xor(vacc[i], 32, 64);
    } else {  // no column of this chunk for this wavefront: fetch the next
#pragma unroll
      for (int i = 0; i < NB4; ++i) {
        const floatx4 v = reinterpret_cast<const floatx4*>(pb1)[i];
        b[4 * i] = v[0];
        b[4 * i + 1] = v[1];
        b[4 * i + 2] = v[2];
        b[4 * i + 3] = v[3];
      }
#pragma unroll
      for (int ks = 4 * NB4; ks < NU; ++ks) b[ks] = pb1[ks];
    }
    src2 = pair_src[i2];
    dst2 = pair_dst[i2];
    if (ch + 1 < cend && o1 != o0) {  // uniform: the next chunk has another operator
      // the destination row is taken before the copy: a wait for a loaded
      // register issued behind a direct copy into LDS waits for all memory
      // operations
      asm volatile("" : "+v"(dst0));
      lds_reads_done_barrier();
      copy_to_lds<N4>(gt + (size_t)o1 * N4, lds4);
      pending = true;
    }
    if (active) {
      // D layout of a 32x32 block: lane l holds column l % 32, rows
      // 8*(v/4) + 4*(l/32) + v%4 in accumulator element v.
      const int64_t row = (col0 + r < n0) ? (int64_t)rhs * n_pairs + dst0 : trash_row;
      float* out = part + row * PSTR;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int r0 = rb * 32 + 8 * q4 + 4 * h;
          if (rb * 32 + 8 * q4 + 8 <= PSTR)  // same for both halves h
            *reinterpret_cast<floatx4*>(out + r0) =
                floatx4{acc[rb][4 * q4], acc[rb][4 * q4 + 1], acc[rb][4 * q4 + 2],
                        acc[rb][4 * q4 + 3]};
        }
      if (LRV > 0) {
        // rows 32*RB .. 32*RB+LRV-1; lanes of both halves hold the sums,
        // half h writes the even/odd pair starting at 2*h
#pragma unroll
        for (int i = 0; i < LRV; i += 2) {
          if (i + 1 < LRV) {
            if (2 * h == i % 4)
              *reinterpret_cast<float2*>(out + 32 * RB + i) = make_float2(vacc[i], vacc[i + 1]);
          } else if (h == 0) {
            out[32 * RB + i] = vacc[i];
          }
        }
      }
    }
    o0 = o1; n0 = n1; dst0 = dst1;
    o1 = o2; n1 = n2; src1 = src2; dst1 = dst2;
  }
}

template <bool F16>
struct Mfma16;
template <>
struct Mfma16<false> {
  typedef bf16x8 vec;
  static __device__ inline floatx16 run(vec a, vec b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma16<true> {
  typedef halfx8 vec;
  static __device__ inline floatx16 run(vec a, vec b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// 32-bit LDS address of a pointer into __shared__ memory.
__device__ inline unsigned lds_address(const float* p) {
  return (unsigned)reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) float*)p);
}

// One transpose step of a wavefront's tile: writes this lane's four 16-byte
// pieces (one column, rows 8 q .. 8 q + 3 for q = 0..3, at `waddr`), then
// reads four pieces 8 tile rows apart (at `raddr`) and waits for them, all
// in one statement. Written out so that the compiler does not make these
// accesses wait for a direct copy into another LDS buffer still in flight.
__device__ inline void transpose_tile(unsigned waddr, unsigned raddr, floatx4 w0, floatx4 w1,
                                      floatx4 w2, floatx4 w3, floatx4 (&v)[4]) {
  static_assert(kTilePitch * 4 * 8 == 1152, "tile row offsets");
  asm volatile(
      "ds_write_b128 %4, %6\n\t"
      "ds_write_b128 %4, %7 offset:32\n\t"
      "ds_write_b128 %4, %8 offset:64\n\t"
      "ds_write_b128 %4, %9 offset:96\n\t"
      "ds_read_b128 %0, %5\n\t"
      "ds_read_b128 %1, %5 offset:1152\n\t"
      "ds_read_b128 %2, %5 offset:2304\n\t"
      "ds_read_b128 %3, %5 offset:3456\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3])
      : "v"(waddr), "v"(raddr), "v"(w0), "v"(w1), "v"(w2), "v"(w3)
      : "memory");
}

// Parameters of operators evaluated in the translation kernel instead of
// read from a table: the integer offsets of the plan and the problem's box
// side, wavenumber and impedance.
struct GenArgs {
  const int32_t* offsets;  // 3 per offset
  double a, k;
  float inv_k;  // 1 / k
  float psi0;   // k eta / (4 pi): |psi| R
};

// Dyadic Green's function of Eq. (5)-(6) at R = (rx, ry, rz): D = psi [I
// c_iso - R^R^ c_rr], psi = -j k eta e^{-jkR} / (4 pi R), c_iso = 1 -
// j/(kR) - 1/(kR)^2, c_rr = 1 - 3j/(kR) - 3/(kR)^2. The distance and the
// phase kR, reduced to [-pi, pi], are taken in FP64, the rest in FP32 (the
// entries are stored as FP32 anyway). Entry 3 p + q goes to out[3 p + q]
// as (re, im); returns the largest |Re|, |Im|.
__device__ inline float dyadic_green(double rx, double ry, double rz, const GenArgs& ga,
                                     float2* out) {
  const double r = sqrt(rx * rx + ry * ry + rz * rz);
  const double kr = ga.k * r;
  const double twopi = 6.283185307179586476925;
  const float x = (float)(kr - twopi * rint(kr * (1.0 / twopi)));
  float sn, cs;
  sincosf(x, &sn, &cs);
  const float ir = (float)(1.0 / r);
  const float rh[3] = {(float)rx * ir, (float)ry * ir, (float)rz * ir};
  // -j (cos kr - j sin kr) = -sin kr - j cos kr
  const float f = ga.psi0 * ir;
  const float pr = -f * sn, pi = -f * cs;
  const float ikr = ir * ga.inv_k, ikr2 = ikr * ikr;
  const float iso_r = 1.f - ikr2, iso_i = -ikr;
  const float rr_r = 1.f - 3.f * ikr2, rr_i = -3.f * ikr;
  float vmax = 0.f;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const int p = e / 3, q = e - 3 * p;
    const float rr = rh[p] * rh[q];
    const float t_r = (p == q ? iso_r : 0.f) - rr * rr_r;
    const float t_i = (p == q ? iso_i : 0.f) - rr * rr_i;
    const float dr = pr * t_r - pi * t_i, di = pr * t_i + pi * t_r;
    out[e] = make_float2(dr, di);
    vmax = fmaxf(vmax, fmaxf(fabsf(dr), fabsf(di)));
  }
  return vmax;
}

// hi / lo 16-bit parts of v (hi = v rounded, lo = the remainder rounded).
template <bool F16>
__device__ inline void split16(float v, unsigned short& hi, unsigned short& lo) {
  if (F16) {
    const __half h = __float2half_rn(v);
    hi = __half_as_ushort(h);
    lo = __half_as_ushort(__float2half_rn(v - __half2float(h)));
  } else {
    hi = (unsigned short)bf16_rne(v);
    lo = (unsigned short)bf16_rne(v - __uint_as_float((unsigned)hi << 16));
  }
}

// The operator image of offset `o` written into LDS by the whole workgroup,
// in the layout of the 16-bit table (planes re, im of NU rows x KHB values;
// the hi half at img, the lo half at img + lo_off): the sites form one
// uniform lattice of step a / n_d, so each of the (2 n_d - 1)^3 lattice
// differences is evaluated once (one thread each, into `blk`) and the
// NU x NU entries are filled from those blocks, one site pair per thread. FP16 forms divide by the
// power of two that brings the largest |Re|, |Im| to [2^14, 2^15), returned
// in `scale` (1 for BF16). Ends with a barrier; `blk` is free afterwards.
template <int NU, bool F16, int NPROD>
__device__ void generate_operator(const GenArgs& ga, int o, unsigned short* img, int lo_off,
                                  float2* blk, float* wmax, float& scale) {
  constexpr int ND = NU == 3 ? 1 : NU == 24 ? 2 : 3;
  static_assert(3 * ND * ND * ND == NU, "operators are generated for n_d 1..3");
  constexpr int SPAN = 2 * ND - 1, NDIFF = SPAN * SPAN * SPAN;
  constexpr int KHB = (NU + 7) & ~7, PLANE = NU * KHB;
  static_assert(NDIFF <= kBlock, "one lattice difference per thread");
  const int t = threadIdx.x;
  const int wx = ga.offsets[3 * o], wy = ga.offsets[3 * o + 1], wz = ga.offsets[3 * o + 2];
  float vmax = 0.f;
  if (t < NDIFF) {
    const int dx = t / (SPAN * SPAN), dy = (t / SPAN) % SPAN, dz = t % SPAN;
    const double step = ga.a / ND;
    vmax = dyadic_green(ga.a * wx + step * (dx - (ND - 1)), ga.a * wy + step * (dy - (ND - 1)),
                        ga.a * wz + step * (dz - (ND - 1)), ga, blk + 9 * t);
  }
  if (F16) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, m, 64));
    if ((t & 63) == 0) wmax[t >> 6] = vmax;
  }
  lds_reads_done_barrier();
  float inv = 1.f;
  scale = 1.f;
  if (F16) {
    const float m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    const int e = m > 0.f ? ilogbf(m) - 14 : 0;
    scale = ldexpf(1.f, e);
    inv = ldexpf(1.f, -e);  // exact power of two
  }
  // one site pair (l, s) per iteration: its 3 x 3 block of the operator
  constexpr int NS = ND * ND * ND;
  for (int q = t; q < NS * NS; q += kBlock) {
    const int l = q / NS, s = q - l * NS;
    const int lx = l / (ND * ND), ly = (l / ND) % ND, lz = l % ND;
    const int sx = s / (ND * ND), sy = (s / ND) % ND, sz = s % ND;
    const int d = ((lx - sx + ND - 1) * SPAN + (ly - sy + ND - 1)) * SPAN + (lz - sz + ND - 1);
    float2 g[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) g[e] = blk[9 * d + e];
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
      for (int be = 0; be < 3; ++be) {
        unsigned short hr, lr, hi_, li_;
        split16<F16>(g[3 * al + be].x * inv, hr, lr);
        split16<F16>(g[3 * al + be].y * inv, hi_, li_);
        const int at = (3 * l + al) * KHB + 3 * s + be;
        img[at] = hr;
        img[PLANE + at] = hi_;
        if (NPROD == 3) {
          img[lo_off + at] = lr;
          img[lo_off + PLANE + at] = li_;
        }
      }
  }
  lds_reads_done_barrier();
}

// Split-precision translation on the 16-bit matrix cores
// (v_mfma_f32_32x32x16_bf16 / _f16, FP32 accumulation). With G = Gh + Gl
// and P = Ph + Pl (h = the value rounded to 16 bits, l = the remainder
// rounded), NPROD = 3 takes the product as Gh Ph + Gh Pl + Gl Ph (the
// dropped Gl Pl term and each split's representation error are about
// 2^-16 relative in BF16, 2^-22 in FP16); NPROD = 1 takes Gh Ph alone
// (about 2^-11 in FP16). In FP16 the operator is stored divided by a
// power of two per offset and each box vector by a power of two per box
// and RHS; a column's FP32 result is multiplied back by both (exact).
//
// Work layout as in translate_mfma_kernel: each workgroup walks a range of
// chunks (up to 128 pairs of one offset); lane l owns column l % 32 and K
// half h = l / 32; a k-step covers 8 consecutive values of each half (KHB =
// NU rounded up to 8, zero padded), read as one 16-byte value per lane from
// the box vector's 64-byte k-step group (the two lanes of a column read
// adjacent 16 bytes); -Gi is a sign flip of the A values; 32-row blocks
// cover all 2*NU rows (padding rows read row 0; their results go to the
// spare row).
//
// Per unit (a chunk, and with WALK one of its right-hand sides): pass 1 runs
// Gh Ph and Gh Pl over all k-steps, pass 2 runs Gl Ph and, k-step by
// k-step, refills the column registers with the next unit's box vector.
// The operator's planes are stored hi half first ([re.hi | im.hi] then
// [re.lo | im.lo]) and copied global -> LDS directly: the first one before
// the loop, each later one (when the next unit has another offset) after
// every wavefront has finished pass 2 and before the partial rows leave, so
// that the copy and the stores are in flight together; the next unit waits
// for the copy alone (the stores issued after it may still be in flight).
// Partial rows leave through a per-wavefront LDS tile: each block is
// written as 4-row pieces per column and read back as 8 columns x 128
// contiguous bytes per store instruction, the destination rows taken once
// per unit from their owner lanes; every wavefront issues the same number
// of stores (absent columns and padding rows go to the spare row), which
// the wait for the copy counts on.
template <int NU, bool F16, int NPROD, bool WALK, bool GEN>
__global__ __launch_bounds__(kBlock, 2) void translate_split_kernel(
    const unsigned short* __restrict__ table, const int32_t* __restrict__ chunks,
    const int32_t* __restrict__ wg_ptr, const int32_t* __restrict__ pair_src,
    const int32_t* __restrict__ pair_dst, const float* __restrict__ P,
    float* __restrict__ part, int64_t n_box, int64_t n_pairs, int64_t trash_row,
    const float* __restrict__ off_scale, const float* __restrict__ box_scale, int nrhs,
    GenArgs ga) {
  typedef typename Mfma16<F16>::vec vec16;
  constexpr int KH = (NU + 3) & ~3;      // FP32 half-length (partial rows)
  constexpr int KHB = (NU + 7) & ~7;     // 16-bit half-length
  constexpr int PLANE = NU * KHB;        // 16-bit values per plane
  constexpr int M = 2 * NU;
  constexpr int RB = (M + 31) / 32;
  constexpr int NGB = KHB / 8;           // k-steps per half
  constexpr int PSTR = 2 * KH;           // partial row (floats)
  constexpr int VSTR = 2 * KHB;          // box vector (floats)
  constexpr int H16 = 2 * PLANE * 2 / 16;                       // 16-byte units per half
  constexpr int HPAD = (H16 + kBlock - 1) / kBlock * kBlock;    // LDS units per half
  constexpr int NLD = HPAD / kBlock;     // copies per thread per half
  constexpr int LO = HPAD * 8;           // lo half, in 16-bit values from the LDS start
  __shared__ uintx4 lds4[(NPROD == 3 ? 2 : 1) * HPAD];
  __shared__ floatx4 tiles4[4][32 * kTilePitch / 4];  // one per wavefront
  __shared__ float gen_max[4];                         // GEN: per-wavefront maxima
  const unsigned short* lds = reinterpret_cast<const unsigned short*>(lds4);

  const int group = xcd_chunk(blockIdx.x, gridDim.x);
  const int cbeg = wg_ptr[group], cend = wg_ptr[group + 1];
  // WALK: the workgroup walks work units v = chunk * nrhs + rhs over its
  // chunks (every right-hand side of a chunk in turn, one staging of the
  // operator for all of them); otherwise one right-hand side per grid row
  const int nv = WALK ? nrhs : 1;
  const int vbeg = cbeg * nv, vend = cend * nv;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;

  // Operator rows of this lane per block: Er rows read re (h = 0) or -im
  // (h = 1); Ei rows read im (h = 0) or re (h = 1). Plane c = 0 re, 1 im.
  int abase[RB];
  unsigned asgn[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int row = rb * 32 + r;
    const bool er = row < NU;
    const int rr = er ? row : (row < M ? row - NU : 0);
    const int c = er ? (h == 1 ? 1 : 0) : (row < M && h == 0 ? 1 : 0);
    abase[rb] = c * PLANE + rr * KHB;
    asgn[rb] = (er && h == 1) ? 0x80008000u : 0u;
  }

  if (cbeg >= cend) return;
  const int col0 = wave * 32;
  const int64_t last = n_pairs - 1;

  // Unconditional memory operations: pair indices one unit ahead, B values
  // one unit ahead (refilled in pass 2), the next operator copied straight
  // into LDS before the partial rows leave.
  auto unit_rhs = [&](int v) { return WALK ? v % nv : (int)blockIdx.y; };
  int o0 = chunks[4 * cbeg], n0 = chunks[4 * cbeg + 2];
  int rhs0 = unit_rhs(vbeg);
  int dst0;
  vec16 bh[NGB], bl[NPROD == 3 ? NGB : 1];
  float bsc0 = 1.f;
  {
    const int64_t i0 = min((int64_t)chunks[4 * cbeg + 1] + col0 + r, last);
    const int src0 = pair_src[i0];
    dst0 = pair_dst[i0];
    // k-step g of a box vector is 64 bytes: hi of both halves, then lo of both
    const vec16* pv = reinterpret_cast<const vec16*>(P + ((int64_t)rhs0 * n_box + src0) * VSTR);
#pragma unroll
    for (int g = 0; g < NGB; ++g) {
      bh[g] = pv[4 * g + h];
      if (NPROD == 3) bl[g] = pv[4 * g + 2 + h];
    }
    // FP16: the scale of the current chunk's column (this lane's source box)
    if (F16) bsc0 = box_scale[(int64_t)rhs0 * n_box + src0];
  }
  const uintx4* gt = reinterpret_cast<const uintx4*>(table);
  constexpr size_t OPU = 4 * PLANE / 8;  // 16-byte units per operator
  unsigned short* const img = reinterpret_cast<unsigned short*>(lds4);
  float2* const blk = reinterpret_cast<float2*>(&tiles4[0][0]);
  float gen_scale = 1.f;  // GEN: the staged operator's power-of-two scale
  int staged = -1;        // GEN: offset of the staged operator
  if (GEN) {
    // the padding columns of every row stay zero (generation writes the
    // first NU of each row only)
    constexpr int PADC = KHB - NU, NH = NPROD == 3 ? 2 : 1;
    constexpr int PC = PADC > 0 ? PADC : 1;  // divisor (no padding: no iterations)
    for (int q = threadIdx.x; q < NH * 2 * NU * PADC; q += kBlock) {
      const int hh = q / (2 * NU * PC), rem = q - hh * 2 * NU * PC;
      const int row = rem / PC;  // plane-major: re rows, then im rows
      img[hh * LO + row * KHB + NU + (rem - row * PC)] = 0;
    }
  } else {
    copy_to_lds<H16>(gt + (size_t)o0 * OPU, lds4);
    if (NPROD == 3) copy_to_lds<H16>(gt + (size_t)o0 * OPU + H16, lds4 + HPAD);
    wait_vmcnt<0>();
    lds_copies_done_barrier();
  }

  bool pending = false;
  for (int v = vbeg; v < vend; ++v) {
    if (GEN) {
      if (o0 != staged) {  // uniform across the workgroup
        lds_reads_done_barrier();  // every wavefront is done with the image and its tile
        generate_operator<NU, F16, NPROD>(ga, o0, img, LO, blk, gen_max, gen_scale);
        staged = o0;
      }
    } else if (pending) {
      // the copy was issued just before the previous unit's RB * 4 stores
      wait_vmcnt<RB * 4>();
      lds_copies_done_barrier();
      pending = false;
    }
    const bool has1 = v + 1 < vend;
    const int c1 = (v + 1) / nv;
    const int rhs1 = has1 ? unit_rhs(v + 1) : rhs0;
    const int o1 = has1 ? chunks[4 * c1] : o0;
    const int b1 = has1 ? chunks[4 * c1 + 1] : 0;
    const int n1 = has1 ? chunks[4 * c1 + 2] : 0;
    const int64_t i1 = min((int64_t)b1 + col0 + r, last);
    const int src1 = pair_src[i1];
    const int dst1 = pair_dst[i1];
    const bool active = col0 < n0;  // wave-uniform

    floatx16 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb] = floatx16{};
    // The passes run at a raised wavefront priority: the other wavefront on
    // the SIMD (another workgroup's) is then mostly in its copy, stores or
    // start, and its instructions are issued around the matrix-core ones.
    __builtin_amdgcn_s_setprio(1);
    if (active) {
      // pass 1: Gh Ph (+ Gh Pl)
#pragma unroll
      for (int g = 0; g < NGB; ++g) {
        vec16 a_h[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          uintx4 ah = *reinterpret_cast<const uintx4*>(lds + abase[rb] + 8 * g);
          ah ^= asgn[rb];
          a_h[rb] = __builtin_bit_cast(vec16, ah);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = Mfma16<F16>::run(a_h[rb], bh[g], acc[rb]);
        if (NPROD == 3) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) acc[rb] = Mfma16<F16>::run(a_h[rb], bl[g], acc[rb]);
        }
      }
    }
    // the next unit's column: its box vector is fetched in pass 2, its FP16
    // scale here
    const vec16* pv1 = reinterpret_cast<const vec16*>(P + ((int64_t)rhs1 * n_box + src1) * VSTR);
    const float bsc1 = F16 ? box_scale[(int64_t)rhs1 * n_box + src1] : 1.f;
    // pass 2: Gl Ph, refilling the registers with the next unit's columns
    // (the test is per k-step so that each refill stays next to its k-step's
    // products instead of being gathered after the pass)
#pragma unroll
    for (int g = 0; g < NGB; ++g) {
      if (NPROD == 3) {
        if (active) {
          vec16 a_l[RB];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            uintx4 al = *reinterpret_cast<const uintx4*>(lds + LO + abase[rb] + 8 * g);
            al ^= asgn[rb];
            a_l[rb] = __builtin_bit_cast(vec16, al);
          }
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) acc[rb] = Mfma16<F16>::run(a_l[rb], bh[g], acc[rb]);
        }
        bl[g] = pv1[4 * g + 2 + h];
      }
      bh[g] = pv1[4 * g + h];
    }
    __builtin_amdgcn_s_setprio(0);
    if (!GEN && has1 && o1 != o0) {  // uniform: the next unit has another operator
      lds_reads_done_barrier();
      copy_to_lds<H16>(gt + (size_t)o1 * OPU, lds4);
      if (NPROD == 3) copy_to_lds<H16>(gt + (size_t)o1 * OPU + H16, lds4 + HPAD);
      pending = true;
    }

    // Every wavefront stores RB * 4 times (absent columns and padding rows
    // go to the spare row), so the wait for the copy above is exact.
    {
      const float sc = F16 ? (GEN ? gen_scale : off_scale[o0]) * bsc0 : 1.f;
      float* tile = reinterpret_cast<float*>(tiles4[wave]);
      float* part_rhs = part + (int64_t)rhs0 * n_pairs * PSTR;
      float* spare = part + trash_row * PSTR;
      const int seg = lane & 7;
      // destination row of the columns this lane stores (c = lane/8 + 8 it)
      int64_t rowoff[4];
      bool cok[4];
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int c = (lane >> 3) + 8 * it;
        rowoff[it] = (int64_t)__shfl(dst0, c, 64) * PSTR;
        cok[it] = c < n0 - col0;
      }
      const unsigned wr = lds_address(tile + r * kTilePitch + 4 * h);
      const unsigned rd = lds_address(tile + (lane >> 3) * kTilePitch + 4 * seg);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        floatx4 w[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
          w[q4] = floatx4{acc[rb][4 * q4], acc[rb][4 * q4 + 1], acc[rb][4 * q4 + 2],
                          acc[rb][4 * q4 + 3]} * sc;
        floatx4 vv[4];
        transpose_tile(wr, rd, w[0], w[1], w[2], w[3], vv);
        const int m = rb * 32 + 4 * seg;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          float* dp = (cok[it] && m + 4 <= PSTR) ? part_rhs + rowoff[it] + m
                                                 : spare + min(m, PSTR - 4);
          *reinterpret_cast<floatx4*>(dp) = vv[it];
        }
      }
    }
    o0 = o1; n0 = n1; dst0 = dst1; rhs0 = rhs1;
    bsc0 = bsc1;
  }
}

// The split-precision translation in rounds of four items per workgroup of
// four wavefronts, so that a wavefront's memory traffic overlaps its own
// matrix-core work. Two workgroups per compute unit with one operator
// buffer each (DOUBLE = false), or one per compute unit with two buffers
// (DOUBLE = true: the next segment's operator is copied during this one):
// * each workgroup walks its rounds (p.rounds); in a round, wavefront w
//   takes one item (up to 32 pairs of one offset, one column each) of the
//   current segment (a run of one offset);
// * a segment's operator is copied straight into LDS (global -> LDS, no
//   registers); with two buffers, the next segment's copy is issued when a
//   segment starts and arrives while that segment runs;
// * pass 1 accumulates Gh Ph (+ Gh Pl) over all k-steps into every 32-row
//   block; pass 2 adds Gl Ph block pair by block pair, so each pair is
//   complete, and its partial rows are stored (through the wavefront's
//   transposing LDS tile), while the next pair computes;
// * the next item's columns are fetched during pass 2.
// Columns past an item's count repeat its last pair (same values stored to
// the same row again), so no store is masked. Per column the arithmetic is
// the same products as translate_split_kernel, accumulated in another order.
template <int NU, bool F16, int NPROD, bool DOUBLE>
__global__ __launch_bounds__(kBlock, DOUBLE ? 1 : 2) void translate_rounds_kernel(
    const unsigned short* __restrict__ table, const int32_t* __restrict__ rounds,
    const int32_t* __restrict__ wg_round_ptr, const int32_t* __restrict__ pair_src,
    const int32_t* __restrict__ pair_dst, const float* __restrict__ P,
    float* __restrict__ part, int64_t n_box, int64_t n_pairs,
    const float* __restrict__ off_scale, const float* __restrict__ box_scale) {
  typedef typename Mfma16<F16>::vec vec16;
  constexpr int KH = (NU + 3) & ~3;
  constexpr int KHB = (NU + 7) & ~7;
  constexpr int PLANE = NU * KHB;
  constexpr int M = 2 * NU;
  constexpr int RB = (M + 31) / 32;
  constexpr int NGB = KHB / 8;
  constexpr int PSTR = 2 * KH;
  constexpr int VSTR = 2 * KHB;
  constexpr int H16 = 2 * PLANE * 2 / 16;
  constexpr int HPAD = (H16 + kBlock - 1) / kBlock * kBlock;
  constexpr int OPB = (NPROD == 3 ? 2 : 1) * HPAD;  // 16-byte units per operator buffer
  constexpr int LO = HPAD * 8;                      // lo half, in 16-bit values
  // rows of the last 32-row block that belong to the partial row
  constexpr int LR = PSTR - 32 * (RB - 1);
  static_assert(LR % 8 == 0 && LR <= 32, "rows of the last block");
  __shared__ uintx4 opbuf0[OPB];
  __shared__ uintx4 opbuf1[DOUBLE ? OPB : 1];
  __shared__ floatx4 tiles4[4][32 * kTilePitch / 4];

  const int group = xcd_chunk(blockIdx.x, gridDim.x);
  const int kbeg = wg_round_ptr[group], kend = wg_round_ptr[group + 1];
  const int rhs = blockIdx.y;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5, seg = lane & 7;

  int abase[RB];
  unsigned asgn[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int row = rb * 32 + r;
    const bool er = row < NU;
    const int rr = er ? row : (row < M ? row - NU : 0);
    const int c = er ? (h == 1 ? 1 : 0) : (row < M && h == 0 ? 1 : 0);
    abase[rb] = c * PLANE + rr * KHB;
    asgn[rb] = (er && h == 1) ? 0x80008000u : 0u;
  }
  if (kbeg >= kend) return;

  const int4* rd = reinterpret_cast<const int4*>(rounds);
  const int64_t last = n_pairs - 1;
  float* tile = reinterpret_cast<float*>(tiles4[wave]);
  float* part_rhs = part + (int64_t)rhs * n_pairs * PSTR;
  auto copy_operator = [&](int o, uintx4* dst) {
    const uintx4* g4 = reinterpret_cast<const uintx4*>(table + (size_t)o * 4 * PLANE);
    copy_to_lds<H16>(g4, dst);
    if (NPROD == 3) copy_to_lds<H16>(g4 + H16, dst + HPAD);
  };
  auto column = [&](const int4& d) {
    return min((int64_t)d.y + min(r, max(d.z - 1, 0)), last);
  };

  // this wavefront's items of rounds k, k+1 (descriptors) and their columns
  int4 d0 = rd[(int64_t)kbeg * 4 + wave];
  int4 d1 = kbeg + 1 < kend ? rd[(int64_t)(kbeg + 1) * 4 + wave] : int4{0, 0, 0, 0};
  const int64_t i0 = column(d0), i1 = column(d1);
  int src0 = pair_src[i0], dst0 = pair_dst[i0];
  int src1 = pair_src[i1], dst1 = pair_dst[i1];
  vec16 bh[NGB], bl[NPROD == 3 ? NGB : 1];
  {
    const vec16* pv = reinterpret_cast<const vec16*>(P + ((int64_t)rhs * n_box + src0) * VSTR);
#pragma unroll
    for (int g = 0; g < NGB; ++g) {
      bh[g] = pv[4 * g + h];
      if (NPROD == 3) bl[g] = pv[4 * g + 2 + h];
    }
  }
  float bsc0 = F16 ? box_scale[(int64_t)rhs * n_box + src0] : 1.f;

  // one round with the current segment's operator in `cur`
  auto round = [&](const uintx4* cur, int k) {
    // Indices two rounds ahead and the next item's scale are requested
    // before this round's stores: a later wait for them then lets the
    // stores stay in flight (vector memory operations complete in order).
    const bool has2 = k + 2 < kend;
    const int4 d2 = has2 ? rd[(int64_t)(k + 2) * 4 + wave] : int4{0, 0, 0, 0};
    const int64_t i2 = column(d2);
    const int src2 = pair_src[i2];
    const int dst2 = pair_dst[i2];
    const float bsc1 = F16 ? box_scale[(int64_t)rhs * n_box + src1] : 1.f;
    const vec16* pv1 = reinterpret_cast<const vec16*>(P + ((int64_t)rhs * n_box + src1) * VSTR);

    if (d0.z > 0) {  // wave-uniform: this wavefront has an item in this round
      const unsigned short* opb = reinterpret_cast<const unsigned short*>(cur);
      const float sc = F16 ? off_scale[d0.x] * bsc0 : 1.f;
      // destination rows of the columns this lane stores: full blocks, lane l
      // takes column l/8 + 8 it, rows 4 (l%8) .. +3; the last block, column
      // l/2, rows 4 (l%2) + 8 it .. +3
      int row_f[4];
#pragma unroll
      for (int it = 0; it < 4; ++it) row_f[it] = __shfl(dst0, (lane >> 3) + 8 * it, 64);
      const int row_l = __shfl(dst0, lane >> 1, 64);
      floatx16 acc[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[rb] = floatx16{};
      auto store_block = [&](int rb) {
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
          *reinterpret_cast<floatx4*>(tile + r * kTilePitch + 8 * q4 + 4 * h) =
              floatx4{acc[rb][4 * q4], acc[rb][4 * q4 + 1], acc[rb][4 * q4 + 2],
                      acc[rb][4 * q4 + 3]} * sc;
        if (rb < RB - 1) {
          floatx4 v[4];
#pragma unroll
          for (int it = 0; it < 4; ++it)
            v[it] = *reinterpret_cast<const floatx4*>(
                tile + ((lane >> 3) + 8 * it) * kTilePitch + 4 * seg);
#pragma unroll
          for (int it = 0; it < 4; ++it)
            *reinterpret_cast<floatx4*>(part_rhs + (int64_t)row_f[it] * PSTR + rb * 32 +
                                        4 * seg) = v[it];
        } else {
          floatx4 v[LR / 8];
#pragma unroll
          for (int it = 0; it < LR / 8; ++it)
            v[it] = *reinterpret_cast<const floatx4*>(tile + (lane >> 1) * kTilePitch +
                                                      4 * (lane & 1) + 8 * it);
#pragma unroll
          for (int it = 0; it < LR / 8; ++it)
            *reinterpret_cast<floatx4*>(part_rhs + (int64_t)row_l * PSTR + rb * 32 +
                                        4 * (lane & 1) + 8 * it) = v[it];
        }
      };

      // pass 1: Gh Ph (+ Gh Pl) into every block
#pragma unroll
      for (int g = 0; g < NGB; ++g) {
        vec16 a_h[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          uintx4 ah = *reinterpret_cast<const uintx4*>(opb + abase[rb] + 8 * g);
          ah ^= asgn[rb];
          a_h[rb] = __builtin_bit_cast(vec16, ah);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = Mfma16<F16>::run(a_h[rb], bh[g], acc[rb]);
        if (NPROD == 3) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) acc[rb] = Mfma16<F16>::run(a_h[rb], bl[g], acc[rb]);
        }
      }
      if (NPROD == 3) {
        // the lo halves of this column are used up: fetch the next item's
#pragma unroll
        for (int g = 0; g < NGB; ++g) bl[g] = pv1[4 * g + 2 + h];
        // pass 2: Gl Ph, two blocks at a time; a finished pair is stored
        // while the next pair computes
#pragma unroll
        for (int q = 0; q < RB; q += 2) {
          const bool two = q + 1 < RB;
#pragma unroll
          for (int g = 0; g < NGB; ++g) {
            uintx4 a0 = *reinterpret_cast<const uintx4*>(opb + LO + abase[q] + 8 * g);
            a0 ^= asgn[q];
            acc[q] = Mfma16<F16>::run(__builtin_bit_cast(vec16, a0), bh[g], acc[q]);
            if (two) {
              uintx4 a1 = *reinterpret_cast<const uintx4*>(opb + LO + abase[q + 1] + 8 * g);
              a1 ^= asgn[q + 1];
              acc[q + 1] = Mfma16<F16>::run(__builtin_bit_cast(vec16, a1), bh[g], acc[q + 1]);
            }
            if (q + 2 >= RB) bh[g] = pv1[4 * g + h];  // last use of bh[g]
          }
          store_block(q);
          if (two) store_block(q + 1);
        }
      } else {
#pragma unroll
        for (int g = 0; g < NGB; ++g) bh[g] = pv1[4 * g + h];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) store_block(rb);
      }
    } else {  // no item for this wavefront in this round: fetch the next
#pragma unroll
      for (int g = 0; g < NGB; ++g) {
        bh[g] = pv1[4 * g + h];
        if (NPROD == 3) bl[g] = pv1[4 * g + 2 + h];
      }
    }
    d0 = d1; d1 = d2;
    src0 = src1; dst0 = dst1; src1 = src2; dst1 = dst2;
    bsc0 = bsc1;
  };

  // segments alternate between the two buffers: even ones read opbuf0 (the
  // next operator is copied into opbuf1), odd ones the reverse
  if constexpr (DOUBLE) {
    // segments alternate between the two buffers: even ones read opbuf0
    // (the next operator is copied into opbuf1), odd ones the reverse
    bool odd = true;
    for (int k = kbeg; k < kend; ++k) {
      if (d0.w & 1) {  // a segment starts (uniform across the workgroup)
        if (k == kbeg) copy_operator(d0.x, opbuf0);
        odd = !odd;
        // this wavefront's copies of the operator (and everything older)
        // have landed; after the barrier every wavefront's have, and every
        // wavefront is done with the other buffer
        wait_vmcnt<0>();
        lds_copies_done_barrier();
        const int next = (d0.w >> 1) - 1;
        if (next >= 0) copy_operator(next, odd ? opbuf0 : opbuf1);
      }
      if (odd) round(opbuf1, k);
      else round(opbuf0, k);
    }
  } else {
    // one buffer: a segment's operator is copied when it starts
    for (int k = kbeg; k < kend; ++k) {
      if (d0.w & 1) {  // a segment starts (uniform across the workgroup)
        if (k != kbeg) lds_reads_done_barrier();  // every wavefront is done with the operator
        copy_operator(d0.x, opbuf0);
        wait_vmcnt<0>();
        lds_copies_done_barrier();
      }
      round(opbuf0, k);
    }
  }
}

// ---------------------------------------------------------------- stage 3

// Complex values of S_j staged in LDS per column batch (81 columns of 81,
// plus one element of alignment slack at each end).
constexpr int kStage = 81 * 81 + 2;

// E_j into LDS (planar padded, 2*kh floats): either the sum of the box's
// partial products (its consecutive rows of the partial buffer, read as
// float4; the row groups' sums are combined through `scratch`) or a
// complex input vector. Ends with a barrier. With PU > 0 the first PU rows
// of each row group are all requested before any is used (rows past the
// box's last one are read clamped and masked out), so they are in flight
// together with the caller's earlier loads; PU = 0 streams the rows.
template <bool FROM_PARTS, int PU>
__device__ inline void gather_E(const float* __restrict__ part,
                                const int32_t* __restrict__ test_ptr, int64_t n_pairs,
                                const float2* __restrict__ Ein, int64_t j, int r,
                                int64_t n_box, int nu, int kh, float4* scratch,
                                float4* Es4) {
  const int t = threadIdx.x;
  if (FROM_PARTS) {
    const int R4 = kh / 2;                     // float4 per partial row
    const int H = kBlock / R4;                 // row groups
    const int g = t % R4, h = t / R4;
    const int p0 = test_ptr[j], p1 = test_ptr[j + 1];
    const float4* pr = reinterpret_cast<const float4*>(part) + (int64_t)r * n_pairs * R4;
    if (h < H) {
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      int p = p0 + h;
      if (PU > 0 && p1 > p0) {  // uniform
        float4 v[PU > 0 ? PU : 1];
#pragma unroll
        for (int i = 0; i < PU; ++i) v[i] = load_once(&pr[(int64_t)min(p + i * H, p1 - 1) * R4 + g]);
#pragma unroll
        for (int i = 0; i < PU; ++i)
          if (p + i * H < p1) {
            acc.x += v[i].x;
            acc.y += v[i].y;
            acc.z += v[i].z;
            acc.w += v[i].w;
          }
        p += PU * H;
      }
#pragma unroll 4
      for (; p < p1; p += H) {
        const float4 v = load_once(&pr[(int64_t)p * R4 + g]);
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
      }
      scratch[h * R4 + g] = acc;
    }
    __syncthreads();
    for (int m4 = t; m4 < R4; m4 += kBlock) {
      float4 s4 = scratch[m4];
      for (int hh = 1; hh < H; ++hh) {
        const float4 v = scratch[hh * R4 + m4];
        s4.x += v.x;
        s4.y += v.y;
        s4.z += v.z;
        s4.w += v.w;
      }
      Es4[m4] = s4;
    }
  } else {
    float* Es = reinterpret_cast<float*>(Es4);
    for (int u = t; u < nu; u += kBlock) {
      const float2 e = Ein[((int64_t)r * n_box + j) * nu + u];
      Es[u] = e.x;
      Es[nu + u] = e.y;
    }
  }
  __syncthreads();
}

// y_j[c0 + c] = sum_u S_j[u, c0 + c] E_j[u] for the ncol columns staged in
// LDS (`shift` slots in). A wavefront takes 16 columns per pass; lane l
// handles column l % 16 and rows u = q, q + 4, q + 8, ... with q = l / 16,
// so the 16 lanes of a quarter read 16 different columns (conflict-free
// 8-byte LDS reads) and the rows of E_j a lane needs are fixed: they are
// held in registers (er/ei, EQ >= ceil(nu / 4) rows per lane).
template <int EQ>
__device__ inline void apply_staged(const float2* stage, int shift, int ncol,
                                    const float (&er)[EQ], const float (&ei)[EQ],
                                    int nu, float2* yb) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int q = lane >> 4;
  for (int cb = wave * 16; cb < ncol; cb += kBlock / 4) {
    const int c = cb + (lane & 15);
    float sr = 0.f, si = 0.f;
    if (c < ncol) {
      const float2* col = stage + shift + c * nu + q;
#pragma unroll
      for (int i = 0; i < EQ; ++i) {
        if (q + 4 * i < nu) {
          const float2 sv = col[4 * i];
          sr = fmaf(sv.x, er[i], fmaf(-sv.y, ei[i], sr));
          si = fmaf(sv.x, ei[i], fmaf(sv.y, er[i], si));
        }
      }
    }
    sr += __shfl_xor(sr, 16, 64);
    si += __shfl_xor(si, 16, 64);
    sr += __shfl_xor(sr, 32, 64);
    si += __shfl_xor(si, 32, 64);
    if (c < ncol && q == 0) yb[c] = make_float2(sr, si);
  }
}

// One workgroup per (test box, rhs): E_j (gather_E), then y_j = T_j E_j.
// mode 0: identity basis (y_j = E_j). mode 1: T_j = S_j^T; S_j is read in
// batches of CB columns, staged in LDS and applied by apply_staged. In a
// batch, slots (float4 = two complex values from the 16-byte aligned
// address at or below the batch start) whose halves both belong to the
// batch are read with indices clamped into that range, so the loads carry
// no branches and all are in flight before any is used; the at most two
// half slots at the ends are read as float2. The first batch is issued
// before E_j is gathered, overlapping the two streams. mode 2: explicit
// column-major T_j, one thread per output row.
// LDS (about 54 KB) allows three workgroups per compute unit; the bound
// lets the compiler keep a whole staged batch in registers. EQ is the
// number of E_j rows each lane keeps (ceil(nu / 4) at most).
template <bool FROM_PARTS, int EQ>
__global__ __launch_bounds__(kBlock, EQ <= 21 ? 3 : 2) void disaggregate_kernel(
    const float* __restrict__ part, const int32_t* __restrict__ test_ptr,
    int64_t n_pairs, const float2* __restrict__ Ein, const int64_t* __restrict__ nb_ptr,
    const float2* __restrict__ S, const float2* __restrict__ T, int mode,
    float2* __restrict__ y, int64_t n_box, int64_t nb_total, int nu, int kh) {
  constexpr int LD = ((kStage + 1) / 2 + kBlock - 1) / kBlock;
  __shared__ float4 Es4[98];                  // E_j, planar padded (2*kh floats)
  __shared__ float4 stage4[(kStage + 1) / 2];  // S_j batch, or gather scratch
  const float* Es = reinterpret_cast<const float*>(Es4);
  const float2* stage = reinterpret_cast<const float2*>(stage4);
  const int64_t j = blockIdx.x;
  const int r = blockIdx.y;
  const int t = threadIdx.x;
  float2* yb = y + (int64_t)r * nb_total;

  if (mode == 0) {
    gather_E<FROM_PARTS, 0>(part, test_ptr, n_pairs, Ein, j, r, n_box, nu,
                            kh, stage4, Es4);
    for (int u = t; u < nu; u += kBlock) yb[j * nu + u] = make_float2(Es[u], Es[nu + u]);
    return;
  }
  const int64_t start = nb_ptr[j];
  const int64_t nb = nb_ptr[j + 1] - start;
  if (mode == 2) {
    gather_E<FROM_PARTS, 0>(part, test_ptr, n_pairs, Ein, j, r, n_box, nu,
                            kh, stage4, Es4);
    const float2* Tb = T + start * nu;
    for (int64_t c = t; c < nb; c += kBlock) {
      float sr = 0.f, si = 0.f;
#pragma unroll 9
      for (int u = 0; u < nu; ++u) {
        const float2 v = Tb[c + nb * u];
        const float er = Es[u], ei = Es[nu + u];
        sr = fmaf(v.x, er, fmaf(-v.y, ei, sr));
        si = fmaf(v.x, ei, fmaf(v.y, er, si));
      }
      yb[start + c] = make_float2(sr, si);
    }
    return;
  }

  // mode 1
  const int CB = (kStage - 2) / nu;            // columns per batch
  if (nb <= 0) {
    gather_E<FROM_PARTS, 0>(part, test_ptr, n_pairs, Ein, j, r, n_box, nu,
                            kh, stage4, Es4);
    return;
  }
  // First batch: its loads are in flight while E_j is gathered.
  {
    const int ncol = (int)min((int64_t)CB, nb);
    const float2* blk = S + start * nu;
    const int shift = (reinterpret_cast<uintptr_t>(blk) & 15) ? 1 : 0;
    const int lim = ncol * nu + shift;
    const int n4 = (lim + 1) / 2;
    const int lo = shift;
    const int hi = (lim & 1) ? n4 - 2 : n4 - 1;
    const float2* s2 = blk - shift;
    const floatx4* s4 = reinterpret_cast<const floatx4*>(s2);
    floatx4 tmp[LD];
#pragma unroll
    for (int it = 0; it < LD; ++it) tmp[it] = s4[min(max(t + it * kBlock, lo), hi)];
    const float2 edge0 = s2[shift ? 1 : 2 * lo];
    const float2 edge1 = s2[(lim & 1) ? 2 * (n4 - 1) : 2 * hi];
    gather_E<FROM_PARTS, 8>(part, test_ptr, n_pairs, Ein, j, r, n_box, nu, kh, stage4, Es4);
    floatx4* stagev = reinterpret_cast<floatx4*>(stage4);
#pragma unroll
    for (int it = 0; it < LD; ++it) {
      const int i = t + it * kBlock;
      if (i >= lo && i <= hi) stagev[i] = tmp[it];
    }
    if (t == 0 && shift) stagev[0] = floatx4{0.f, 0.f, edge0.x, edge0.y};
    if (t == 1 && (lim & 1)) stagev[n4 - 1] = floatx4{edge1.x, edge1.y, 0.f, 0.f};
    float er[EQ], ei[EQ];  // this lane's rows of E_j (see apply_staged)
    const int q = (t & 63) >> 4;
#pragma unroll
    for (int i = 0; i < EQ; ++i) {
      const int u = min(q + 4 * i, nu - 1);
      er[i] = Es[u];
      ei[i] = Es[nu + u];
    }
    __syncthreads();
    apply_staged<EQ>(stage, shift, ncol, er, ei, nu, yb + start);
  }
  // Boxes with more than CB functions: further batches are copied straight
  // into LDS and applied with E_j read from LDS (rare).
  for (int64_t c0 = CB; c0 < nb; c0 += CB) {
    __syncthreads();  // previous batch fully consumed
    const int ncol = (int)min((int64_t)CB, nb - c0);
    const float2* blk = S + (start + c0) * nu;
    const int shift = (reinterpret_cast<uintptr_t>(blk) & 15) ? 1 : 0;
    const int lim = ncol * nu + shift;
    const int n4 = (lim + 1) / 2;
    const int lo = shift;
    const int hi = (lim & 1) ? n4 - 2 : n4 - 1;
    const float2* s2 = blk - shift;
    const floatx4* s4 = reinterpret_cast<const floatx4*>(s2);
    floatx4* stagev = reinterpret_cast<floatx4*>(stage4);
    for (int i = lo + t; i <= hi; i += kBlock) stagev[i] = s4[i];
    if (t == 0 && shift) {
      const float2 v = s2[1];
      stagev[0] = floatx4{0.f, 0.f, v.x, v.y};
    }
    if (t == 1 && (lim & 1)) {
      const float2 v = s2[2 * (n4 - 1)];
      stagev[n4 - 1] = floatx4{v.x, v.y, 0.f, 0.f};
    }
    __syncthreads();
    const int quarter = t & 3;
    for (int cb = 0; cb < ncol; cb += kBlock / 4) {
      const int c = cb + (t >> 2);
      float sr = 0.f, si = 0.f;
      if (c < ncol) {
        const float2* col = stage + shift + c * nu;
        for (int u = quarter; u < nu; u += 4) {
          const float2 sv = col[u];
          sr = fmaf(sv.x, Es[u], fmaf(-sv.y, Es[nu + u], sr));
          si = fmaf(sv.x, Es[nu + u], fmaf(sv.y, Es[u], si));
        }
      }
      sr += __shfl_xor(sr, 1, 64);
      si += __shfl_xor(si, 1, 64);
      sr += __shfl_xor(sr, 2, 64);
      si += __shfl_xor(si, 2, 64);
      if (c < ncol && quarter == 0) yb[start + c0 + c] = make_float2(sr, si);
    }
  }
}

// Stage 3 with one wavefront per box (E_j from the partial rows, N_u <= 84;
// T_j = S_j^T, or y_j = E_j with IDENT): no workgroup barriers on the box's
// path. The wavefront serves a block of up to RB right-hand sides. For each,
// lane l < R4 sums float4 l of the box's partial rows (16 rows in flight);
// the sums go to the wavefront's own LDS slot (672 bytes per vector) and
// come back as this lane's rows of E_j; then four columns of S_j per pass,
// 16 lanes per column, read from global memory once for the RB vectors and
// reduced across the 16 lanes by shuffles. Same arithmetic as
// disaggregate_kernel except the order of the sums.
template <int EQ, bool IDENT, int RB>
__global__ __launch_bounds__(kBlock) void disaggregate_wave_kernel(
    const float* __restrict__ part, const int32_t* __restrict__ test_ptr, int64_t n_pairs,
    const int64_t* __restrict__ nb_ptr, const float2* __restrict__ S, float2* __restrict__ y,
    int64_t n_box, int64_t nb_total, int nu, int kh, int nrhs) {
  constexpr int RU = 16;  // partial rows in flight per lane
  __shared__ float4 Es4[kBlock / 64][RB][42];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (j >= n_box) return;  // whole wavefronts; no barriers below
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);  // >= 1
  const int R4 = kh / 2;  // float4 per partial row (<= 42)
  const int p0 = test_ptr[j], p1 = test_ptr[j + 1];
  for (int qr = 0; qr < nr; ++qr) {
    const int r = r0 + qr;
    const float4* pr = reinterpret_cast<const float4*>(part) + (int64_t)r * n_pairs * R4;
    if (lane < R4) {
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int p = p0; p < p1; p += RU) {
        float4 v[RU];
#pragma unroll
        for (int i = 0; i < RU; ++i)
          v[i] = load_once(&pr[(int64_t)min(p + i, p1 - 1) * R4 + lane]);
#pragma unroll
        for (int i = 0; i < RU; ++i)
          if (p + i < p1) {
            acc.x += v[i].x;
            acc.y += v[i].y;
            acc.z += v[i].z;
            acc.w += v[i].w;
          }
      }
      if (IDENT) {  // y_j = E_j: this lane's four positions of [Er | Ei]
        float2* yj = y + (int64_t)r * nb_total + j * nu;
        const float a4[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int pos = 4 * lane + k;
          if (pos < nu) yj[pos].x = a4[k];
          else if (pos < 2 * nu) yj[pos - nu].y = a4[k];
        }
      } else {
        Es4[wave][qr][lane] = acc;
      }
    }
  }
  if (IDENT) return;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  // 16 lanes per column: lane group cs = lane / 16 takes column c0 + cs and
  // lane q = lane % 16 rows q, q + 16, ...; each load instruction reads four
  // whole 128-byte lines of S_j
  constexpr int RQ = (EQ * 4 + 15) / 16;  // rows per lane (N_u <= 4 EQ)
  const int q = lane & 15, cs = lane >> 4;
  float er[RB][RQ], ei[RB][RQ];
#pragma unroll
  for (int qr = 0; qr < RB; ++qr) {
    // vectors past the last one repeat it; their results are not stored
    const float* Es = reinterpret_cast<const float*>(Es4[wave][min(qr, nr - 1)]);
#pragma unroll
    for (int i = 0; i < RQ; ++i) {
      const int u = min(q + 16 * i, nu - 1);
      er[qr][i] = Es[u];
      ei[qr][i] = Es[nu + u];
    }
  }
  const int64_t start = nb_ptr[j];
  const int64_t nb = nb_ptr[j + 1] - start;
  const float2* Sb = S + start * nu;
  for (int64_t c0 = 0; c0 < nb; c0 += 4) {
    const int64_t c = c0 + cs;
    const float2* col = Sb + min(c, nb - 1) * nu;
    float2 sv[RQ];
#pragma unroll
    for (int i = 0; i < RQ; ++i) sv[i] = col[min(q + 16 * i, nu - 1)];
#pragma unroll
    for (int qr = 0; qr < RB; ++qr) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int i = 0; i < RQ; ++i)
        if (q + 16 * i < nu) {
          sr = fmaf(sv[i].x, er[qr][i], fmaf(-sv[i].y, ei[qr][i], sr));
          si = fmaf(sv[i].x, ei[qr][i], fmaf(sv[i].y, er[qr][i], si));
        }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o, 64);
        si += __shfl_xor(si, o, 64);
      }
      if (qr < nr && c < nb && q == 0)
        y[(int64_t)(r0 + qr) * nb_total + start + c] = make_float2(sr, si);
    }
  }
}

// Launch with the stage's timing events when it has them.
#define UBF_LAUNCH(EV, KERNEL, GRID, BLOCK, STREAM, ...)                                 \
  do {                                                                                  \
    if (EV)                                                                             \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, (EV)->start, (EV)->stop, 0, \
                            __VA_ARGS__);                                               \
    else                                                                                \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, __VA_ARGS__);                  \
  } while (0)

// A stage with nothing to launch still completes its events.
int record_empty(const StageEvents* ev, hipStream_t s) {
  if (!ev) return 0;
  hipError_t e = hipEventRecord(ev->start, s);
  if (e == hipSuccess) e = hipEventRecord(ev->stop, s);
  return (int)e;
}

int grid_for(int64_t total) {
  const int64_t g = (total + kBlock - 1) / kBlock;
  return (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

}  // namespace

bool translate_uses_mfma(const Plan& p) {
  return p.nu == 81 || p.nu == 24 || p.nu == 3;
}

int launch_pack(const Plan& p, const void* x, float* P, int nrhs, void* stream,
                const StageEvents* ev) {
  const int64_t rows = (int64_t)nrhs * p.n_box;
  if (p.fp16()) {
    UBF_LAUNCH(ev, pack_f16_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(kBlock),
               (hipStream_t)stream, (const float2*)x, P, p.d_box_scale, p.nu, p.khb, rows);
    return (int)hipGetLastError();
  }
  UBF_LAUNCH(ev, pack_kernel, dim3(grid_for(rows * (p.split() ? p.khb : p.kh))), dim3(kBlock),
             (hipStream_t)stream, (const float2*)x, P, rows, p.nu, p.kh, p.khb,
             p.split() ? 1 : 0);
  return (int)hipGetLastError();
}

int launch_unpack(const Plan& p, const float* P, void* out, int nrhs, void* stream) {
  const int64_t rows = (int64_t)nrhs * p.n_box;
  hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(rows * p.nu)), dim3(kBlock), 0,
                     (hipStream_t)stream, P, (float2*)out, rows, p.nu, p.kh, p.khb,
                     p.fp16() ? 2 : (p.split() ? 1 : 0), p.d_box_scale);
  return (int)hipGetLastError();
}

int launch_aggregate(const Plan& p, const void* x, float* P, int nrhs, void* stream,
                     const StageEvents* ev) {
  if (!p.has_basis) return launch_pack(p, x, P, nrhs, stream, ev);
  // S_i is read once per block of right-hand sides
  const int mode = p.fp16() ? 2 : (p.split() ? 1 : 0);
#define UBF_AGG(RB)                                                                        \
  UBF_LAUNCH(ev, aggregate_kernel<RB>, dim3((unsigned)p.n_box, (nrhs + RB - 1) / RB),      \
             dim3(kBlock), (hipStream_t)stream, (const float2*)x, p.d_nb_ptr,              \
             (const float2*)p.d_S, P, p.n_box, p.nb_total(), p.nu, p.kh, p.khb, mode,       \
             p.d_box_scale, nrhs)
  if (nrhs == 1) UBF_AGG(1); else if (nrhs == 2) UBF_AGG(2); else UBF_AGG(4);
#undef UBF_AGG
  return (int)hipGetLastError();
}

int launch_translate(const Plan& p, const float* P, float* part, int nrhs,
                     void* stream, const StageEvents* ev) {
  const int nch = (int)p.n_chunks();
  hipStream_t s = (hipStream_t)stream;
  if (nch == 0) return record_empty(ev, s);
  const dim3 groups((unsigned)p.n_groups(), nrhs);
  const int64_t trash = (int64_t)p.max_nrhs * p.n_pairs();
  if (p.split()) {
    const unsigned short* tb = reinterpret_cast<const unsigned short*>(p.d_table);
    const int sk = p.split_kernel;
    const bool walk = sk == kSplitChunksWalk && nrhs > 1;
    const dim3 cgrid((unsigned)p.n_groups(), walk ? 1 : nrhs);
    const dim3 rgrid((unsigned)p.n_round_groups(), nrhs);
    if (p.gen_ops && (sk == kSplitRounds || sk == kSplitRoundsDouble))
      return (int)hipErrorInvalidValue;  // rejected by the schedule calls
    const GenArgs ga{p.d_offsets, p.a, p.k, (float)(1.0 / p.k),
                     (float)(p.k * p.eta / (4.0 * 3.14159265358979323846))};
#define UBF_SPLIT_CHUNKS(NU, F16, NPROD, WALK)                                                 \
  do {                                                                                         \
    if (p.gen_ops)                                                                             \
      UBF_LAUNCH(ev, (translate_split_kernel<NU, F16, NPROD, WALK, true>), cgrid, dim3(kBlock), \
                 s, tb, p.d_chunks, p.d_wg_ptr, p.d_pair_src, p.d_pair_dst, P, part, p.n_box,  \
                 p.n_pairs(), trash, p.d_off_scale, p.d_box_scale, nrhs, ga);                  \
    else                                                                                       \
      UBF_LAUNCH(ev, (translate_split_kernel<NU, F16, NPROD, WALK, false>), cgrid, dim3(kBlock), \
                 s, tb, p.d_chunks, p.d_wg_ptr, p.d_pair_src, p.d_pair_dst, P, part, p.n_box,  \
                 p.n_pairs(), trash, p.d_off_scale, p.d_box_scale, nrhs, ga);                  \
  } while (0)
#define UBF_SPLIT(NU, F16, NPROD)                                                              \
  do {                                                                                         \
    if (sk == kSplitRounds || sk == kSplitRoundsDouble) {                                      \
      if (sk == kSplitRoundsDouble)                                                            \
        UBF_LAUNCH(ev, (translate_rounds_kernel<NU, F16, NPROD, true>), rgrid, dim3(kBlock), s,  \
                   tb, p.d_rounds, p.d_wg_round_ptr, p.d_pair_src, p.d_pair_dst, P, part,      \
                   p.n_box, p.n_pairs(), p.d_off_scale, p.d_box_scale);                        \
      else                                                                                     \
        UBF_LAUNCH(ev, (translate_rounds_kernel<NU, F16, NPROD, false>), rgrid, dim3(kBlock), s, \
                   tb, p.d_rounds, p.d_wg_round_ptr, p.d_pair_src, p.d_pair_dst, P, part,      \
                   p.n_box, p.n_pairs(), p.d_off_scale, p.d_box_scale);                        \
    } else if (walk) {                                                                         \
      UBF_SPLIT_CHUNKS(NU, F16, NPROD, true);                                                  \
    } else {                                                                                   \
      UBF_SPLIT_CHUNKS(NU, F16, NPROD, false);                                                 \
    }                                                                                          \
  } while (0)
#define UBF_SPLIT_NU(F16, NPROD)                           \
  switch (p.nu) {                                          \
    case 81: UBF_SPLIT(81, F16, NPROD); break;             \
    case 24: UBF_SPLIT(24, F16, NPROD); break;             \
    case 3: UBF_SPLIT(3, F16, NPROD); break;               \
    default: return (int)hipErrorInvalidValue; /* rejected at plan creation */ \
  }
    if (p.precision == 1) {
      UBF_SPLIT_NU(false, 3);
    } else if (p.precision == 2) {
      UBF_SPLIT_NU(true, 3);
    } else {
      UBF_SPLIT_NU(true, 1);
    }
#undef UBF_SPLIT_NU
#undef UBF_SPLIT
#undef UBF_SPLIT_CHUNKS
    return (int)hipGetLastError();
  }
  switch (p.nu) {
    case 81:
      UBF_LAUNCH(ev, translate_mfma_kernel<81>, groups, dim3(kBlock), s, p.d_table, p.d_chunks,
                 p.d_wg_ptr, p.d_pair_src, p.d_pair_dst, P, part, p.n_box, p.n_pairs(), trash);
      break;
    case 24:
      UBF_LAUNCH(ev, translate_mfma_kernel<24>, groups, dim3(kBlock), s, p.d_table, p.d_chunks,
                 p.d_wg_ptr, p.d_pair_src, p.d_pair_dst, P, part, p.n_box, p.n_pairs(), trash);
      break;
    case 3:
      UBF_LAUNCH(ev, translate_mfma_kernel<3>, groups, dim3(kBlock), s, p.d_table, p.d_chunks,
                 p.d_wg_ptr, p.d_pair_src, p.d_pair_dst, P, part, p.n_box, p.n_pairs(), trash);
      break;
    default:
      // every N_u of n_d 1..4 has a matrix-core kernel (192 goes to the
      // staged one); anything else was rejected at plan creation
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_disaggregate(const Plan& p, bool from_parts, const float* part,
                        const void* E, void* y, int nrhs, void* stream,
                        bool identity, const StageEvents* ev) {
  const int mode = (identity || !p.has_basis) ? 0 : (p.d_T ? 2 : 1);
  const int64_t nb_total = mode == 0 ? p.n_box * (int64_t)p.nu : p.nb_total();
  const dim3 grid((unsigned)p.n_box, nrhs);
  hipStream_t s = (hipStream_t)stream;
  const bool small = p.nu <= 84;  // at most 21 rows of E_j per lane
#define UBF_DISAGG(PARTS, EQ)                                                     \
  UBF_LAUNCH(ev, (disaggregate_kernel<PARTS, EQ>), grid, dim3(kBlock), s, part,        \
             p.d_test_ptr, p.n_pairs(), (const float2*)E, p.d_nb_ptr,                 \
             (const float2*)p.d_S, (const float2*)p.d_T, mode, (float2*)y, p.n_box,    \
             nb_total, p.nu, p.kh)
  // One wavefront per box while a box has up to a few hundred partial rows
  // on average (interaction lists: tens); with thousands per box (FULL far
  // sets) the row sums want a whole workgroup per box.
  const bool few_rows = p.n_pairs() <= 256 * p.n_box;
  // When the boxes fill about two rounds of the chip (up to 16 resident
  // wavefronts per CU), one wavefront per workgroup lets the dispatcher
  // spread them evenly (with four per workgroup a quarter of the CUs of the
  // 3,338-box shell received 16 boxes and the rest 12, and set the time).
  // Larger launches keep four per workgroup: over many rounds the dynamic
  // dispatch balances by itself, and a million one-wavefront workgroups
  // cost a little more to dispatch (1% on the 314,171-box, 4-RHS batch).
  // With T_j = S_j^T a wavefront serves up to four right-hand sides, so
  // that S_j is read once for them; the identity basis has no S_j to share.
  const int rb = (mode == 1 && nrhs > 1) ? (nrhs == 2 ? 2 : 4) : 1;
  const int64_t nrb = (nrhs + rb - 1) / rb;
  const int wpg = (int64_t)p.n_box * nrb <= 8192 ? 1 : kBlock / 64;
  const dim3 wgrid((unsigned)((p.n_box + wpg - 1) / wpg), (unsigned)nrb), wblock(64 * wpg);
#define UBF_WAVE(IDENT, RB)                                                                \
  UBF_LAUNCH(ev, (disaggregate_wave_kernel<21, IDENT, RB>), wgrid, wblock, s, part,        \
             p.d_test_ptr, p.n_pairs(), p.d_nb_ptr, (const float2*)p.d_S, (float2*)y,     \
             p.n_box, nb_total, p.nu, p.kh, nrhs)
  if (from_parts && mode == 1 && small && few_rows) {
    if (rb == 1) UBF_WAVE(false, 1); else if (rb == 2) UBF_WAVE(false, 2); else UBF_WAVE(false, 4);
  } else if (from_parts && mode == 0 && small && few_rows) {
    UBF_WAVE(true, 1);
  } else if (from_parts) {
    if (small) UBF_DISAGG(true, 21); else UBF_DISAGG(true, 49);
  } else {
    if (small) UBF_DISAGG(false, 21); else UBF_DISAGG(false, 49);
  }
#undef UBF_WAVE
#undef UBF_DISAGG
  return (int)hipGetLastError();
}

}  // namespace ubf

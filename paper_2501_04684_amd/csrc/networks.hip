// Stage 2 with the box vectors staged in LDS: translation by complex-valued
// fully connected networks (Sec. 3, Fig. 5) and, for box sizes whose
// columns do not fit in registers, the operator-table product (Eq. 13).
//
// Networks:
// the network of a translation vector w stands in for the product G_w P_i of
// Eq. 13, and stage 3 is unchanged. For a source box vector x (3N_d complex
// values) with s = ||x||_inf (largest modulus) the pair's contribution is
//   s * (W2 CReLU(W1 (x / s) + b1) + b2),
// CReLU acting on real and imaginary parts separately; a zero vector gives
// zero. Both layers run on v_mfma_f32_32x32x2_f32 as real products, each
// MFMA k-step pairing a real K value (lane half 0) with the imaginary one
// (lane half 1):
//   [hr; hi] = [[W1r, -W1i], [W1i, W1r]] [xr; xi]   M = 2*HP, K = 2*NU
//   [Er; Ei] = [[W2r, -W2i], [W2i, W2r]] [hr; hi]   M = 2*NU, K = 2*HP
// with HP = the hidden width rounded up to 32 (hidden units past the
// network's width are zero). s is taken from the staged box vector in
// LDS; the division by s is applied to the layer-1 accumulators and the
// product by s to the layer-2 results, so the staged box vectors are used
// as they are.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "networks.hpp"

namespace ubf {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kBlock = 256;

// Network image of one offset, in floats. The weights are stored in the
// matrix-core fragment order of the kernel below (sign of -W1i / -W2i
// included), so that a wavefront's 16-byte loads of one group of four
// k-steps are 1 KB contiguous:
//   W1 fragments [2 HB row blocks][KH/4 groups][64 lanes][4]: row block rb of
//     [[W1r, -W1i], [W1i, W1r]] (rows: real then imaginary hidden units, HP
//     each), lane l = row l % 32 of the block and input half l / 32
//   b1 (re, im)  [2][HP]
//   W2 fragments [OB row blocks][HP/4 groups][64 lanes][4]: row block ob of
//     [[W2r, -W2i], [W2i, W2r]] (rows: Er then Ei, N_u each), lane l = row
//     l % 32 and hidden half l / 32
//   b2 (re, im)  [2][KH]
// Entries past the network's width, N_u or 2 N_u rows are zero.
__host__ __device__ constexpr int64_t image_floats(int nu, int kh, int hp) {
  return (2LL * hp / 32) * (kh / 4) * 256 + 2LL * hp +
         (int64_t)((2 * nu + 31) / 32) * (hp / 4) * 256 + 2LL * kh;
}

// Value of the real form [[Xr, -Xi], [Xi, Xr]] at a row of the real
// (im_row false) or imaginary part and column half h, from the entry c.
__device__ inline float real_form(float2 c, bool im_row, int h) {
  return !im_row ? (h == 0 ? c.x : -c.y) : (h == 0 ? c.y : c.x);
}

// Caller layout (complex64, offsets in plan order): W1 [n_off][H][NU],
// b1 [n_off][H], W2 [n_off][NU][H], b2 [n_off][NU].
__global__ __launch_bounds__(kBlock) void network_pack_kernel(
    const float2* __restrict__ W1, const float2* __restrict__ b1,
    const float2* __restrict__ W2, const float2* __restrict__ b2, float* __restrict__ img,
    int64_t n_off, int nu, int kh, int hp, int hidden) {
  const int64_t nf = image_floats(nu, kh, hp);
  const int g1 = kh / 4, g2 = hp / 4, hb = hp / 32;
  const int64_t w1 = (int64_t)(2 * hb) * g1 * 256, bb1 = 2LL * hp;
  const int64_t w2 = (int64_t)((2 * nu + 31) / 32) * g2 * 256;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_off * nf;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = t / nf;
    int64_t i = t - o * nf;
    float v = 0.f;
    if (i < w1) {
      const int j = (int)(i & 3), l = (int)((i >> 2) & 63);
      const int64_t bg = i >> 8;
      const int g = (int)(bg % g1), rb = (int)(bg / g1);
      const int row = rb * 32 + (l & 31), h = l >> 5, k = 4 * g + j;
      const bool im_row = row >= hp;
      const int m = im_row ? row - hp : row;
      if (m < hidden && k < nu) v = real_form(W1[(o * hidden + m) * nu + k], im_row, h);
    } else if ((i -= w1) < bb1) {
      const int64_t plane = i / hp, m = i % hp;
      if (m < hidden) {
        const float2 c = b1[o * hidden + m];
        v = plane ? c.y : c.x;
      }
    } else if ((i -= bb1) < w2) {
      const int j = (int)(i & 3), l = (int)((i >> 2) & 63);
      const int64_t bg = i >> 8;
      const int g = (int)(bg % g2), ob = (int)(bg / g2);
      const int row = ob * 32 + (l & 31), h = l >> 5, m = 4 * g + j;
      if (row < 2 * nu && m < hidden) {
        const bool im_row = row >= nu;
        const int u = im_row ? row - nu : row;
        v = real_form(W2[(o * nu + u) * hidden + m], im_row, h);
      }
    } else {
      i -= w2;
      const int64_t plane = i / kh, u = i % kh;
      if (u < nu) {
        const float2 c = b2[o * nu + u];
        v = plane ? c.y : c.x;
      }
    }
    img[t] = v;
  }
}

// acc[i] += A_i B for the PER row blocks a wavefront owns, over G groups of
// four k-steps: per group one 16-byte A load per block and lane (fragment
// order: arow[i] points at the lane's piece of group 0, the next group is
// 64 pieces on) and one 16-byte B load from LDS shared by all blocks;
// consecutive MFMAs go to different blocks' accumulators. The group count
// is G, or ng where it is given (a run-time count of at most G). The loop
// is unrolled U times: measured best at two for the network kernel and at
// one (rolled) for the operator-table kernel, whose three row blocks per
// wavefront already hold three loads in flight.
template <int PER, int G, int U>
__device__ inline void rowblock_products(floatx16 (&acc)[PER], const floatx4* const (&arow)[PER],
                                         const floatx4* brow, int ng = G) {
#pragma unroll U
  for (int g = 0; g < ng; ++g) {
    const floatx4 b = brow[g];
    floatx4 a[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) a[i] = arow[i][g * 64];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int i = 0; i < PER; ++i)
        acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][kk], b[kk], acc[i], 0, 0, 0);
  }
}

// acc += A B for one row block, the loads of group g + D issued before the
// products of group g (a ring of D + 1 register groups), so that loads stay
// in flight across groups; the products are those of rowblock_products in
// the same order. Measured 2 us faster than the two-way unrolled loop for
// layer 1 of the network kernel (64.4 against 62.8 us).
template <int G, int D>
__device__ inline void rowblock_pipelined(floatx16& acc, const floatx4* arow, const floatx4* brow) {
  static_assert(G >= D, "the prologue loads D groups");
  floatx4 a[D + 1], b[D + 1];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    a[d] = arow[d * 64];
    b[d] = brow[d];
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g + D < G) {
      a[(g + D) % (D + 1)] = arow[(g + D) * 64];
      b[(g + D) % (D + 1)] = brow[g + D];
    }
    const floatx4 ac = a[g % (D + 1)], bc = b[g % (D + 1)];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[kk], bc[kk], acc, 0, 0, 0);
  }
}

// Work item of this workgroup: consecutive items (the 32-pair pieces of an
// offset's pairs, which share their weights) go to the same XCD, whose L2
// then fetches those weights once, and every XCD gets the same number of
// items. The hardware deals workgroups to the 8 XCDs round robin; the grid
// is a multiple of 8.
__device__ inline int xcd_item(int bid, int grid) { return (bid & 7) * (grid >> 3) + (bid >> 3); }

// Column staging of one work item: the source box vectors (planar padded,
// [re | im] of KH floats each) of pairs first .. first + ncol - 1 go to LDS
// columns of pitch XP floats, columns past ncol zero. With PASSES = 2 the k
// range is staged in two halves: pass p holds floats [p KH/2, (p + 1) KH/2)
// of the real and of the imaginary part ([re | im] of KH/2 floats), which
// halves the LDS a workgroup needs. The index loads are made once; each
// pass issues all of a thread's vector loads before its LDS writes, so the
// loads overlap instead of forming one chain per piece.
template <int KH, int XP, int PASSES>
struct ColumnStager {
  static constexpr int KP = KH / PASSES;                 // floats of a part per pass
  static constexpr int Q = 2 * KP / 4;                   // 16-byte pieces per column
  static constexpr int IT = (32 * Q + kBlock - 1) / kBlock;  // pieces per thread
  static_assert(KP % 4 == 0 && XP >= 2 * KP, "pass width");
  int src[IT];

  __device__ ColumnStager(const int32_t* __restrict__ pair_src, int first, int ncol) {
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int c = (threadIdx.x + k * kBlock) / Q;
      src[k] = pair_src[first + min(c, ncol - 1)];
    }
  }

  __device__ void stage(floatx4* xs4, const float* __restrict__ Pr, int ncol, int pass) const {
    floatx4 v[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int i = threadIdx.x + k * kBlock;
      const int q = min(i % Q, Q - 1);
      const int part = q / (Q / 2), qq = q - part * (Q / 2);
      v[k] = reinterpret_cast<const floatx4*>(Pr + (int64_t)src[k] * 2 * KH + part * KH +
                                              pass * KP)[qq];
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int i = threadIdx.x + k * kBlock;
      const int c = i / Q, q = i - c * Q;
      if (i < 32 * Q) xs4[c * (XP / 4) + q] = c < ncol ? v[k] : floatx4{0.f, 0.f, 0.f, 0.f};
    }
  }
};

// Passes of the column staging: two where a k half is a whole number of
// four-float groups and the single pass would need more than 32 KB of LDS.
__host__ __device__ constexpr int staging_passes(int kh) {
  return (kh % 8 == 0 && 32 * (2 * kh + 4) * 4 > 32768) ? 2 : 1;
}

// Work item k of this workgroup (XCD-aware, see xcd_item); false for the
// grid's padding.
__device__ inline bool load_item(const int32_t* __restrict__ items, int n_items, int& o,
                                 int& first, int& ncol) {
  const int k = xcd_item(blockIdx.x, gridDim.x);
  if (k >= n_items) return false;
  const int4 it = reinterpret_cast<const int4*>(items)[k];
  o = it.x;
  first = it.y;
  ncol = it.z;
  return true;
}

// One workgroup per work item (up to 32 pairs of one offset, XCD-aware);
// at N_u = 192 the LDS of the two-pass staging lets five share a CU, so
// that the items of a product run in one round. The source box vectors are
// staged in LDS; wavefront w computes layer-1 row blocks w, w + 4, ... (A
// from the network image in fragment order, B from LDS), over the k range
// of each staging pass in turn; after a barrier it writes bias + CReLU into
// the hidden tile, which reuses the staged vectors' LDS, and after another
// barrier computes layer-2 row blocks w, w + 4, ... the same way. Lane l owns pair column
// l % 32; its 4-row pieces of each output block go to the pair's partial
// row, whose positions are the output rows [Er | Ei].
template <int NU, int HB>
__global__ __launch_bounds__(kBlock, 5) void translate_cvfcnn_kernel(
    const float* __restrict__ net, const int32_t* __restrict__ items,
    const int32_t* __restrict__ pair_src, const int32_t* __restrict__ pair_dst,
    const float* __restrict__ P, float* __restrict__ part, int64_t n_box, int64_t n_pairs,
    int hidden, int n_items) {
  constexpr int KH = (NU + 3) & ~3;
  constexpr int HP = 32 * HB;
  constexpr int64_t NF = image_floats(NU, KH, HP);
  constexpr int B1_OFF = 2 * HB * (KH / 4) * 256;
  constexpr int W2_OFF = B1_OFF + 2 * HP;
  constexpr int B2_OFF = W2_OFF + ((2 * NU + 31) / 32) * (HP / 4) * 256;
  constexpr int PASSES = staging_passes(KH);
  constexpr int KP = KH / PASSES;
  constexpr int XP = 2 * KP + 4;     // LDS pitch of a staged box vector
  constexpr int HPT = 2 * HP + 4;    // LDS pitch of a hidden column
  constexpr int OB = (2 * NU + 31) / 32;
  constexpr int PSTR = 2 * KH;
  // the hidden tile reuses the staged vectors' LDS once layer 1 has read them
  constexpr int TILE = 32 * (XP > HPT ? XP : HPT);
  __shared__ floatx4 xs4[TILE / 4];
  __shared__ float col_scale[32];
  __shared__ float bias[2 * HP + 2 * KH];  // b1 (re, im), then b2 (re, im)
  float* xs = reinterpret_cast<float*>(xs4);
  float* hs = xs;

  int o, first, ncol;
  if (!load_item(items, n_items, o, first, ncol)) return;  // grid padding
  const int rhs = blockIdx.y;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int r = lane & 31, h = lane >> 5;
  const float* no = net + (size_t)o * NF;
  const float* Pr = P + (int64_t)rhs * n_box * 2 * KH;

  const ColumnStager<KH, XP, PASSES> stager(pair_src, first, ncol);
  stager.stage(xs4, Pr, ncol, 0);
  for (int i = t; i < 2 * HP + 2 * KH; i += kBlock)
    bias[i] = i < 2 * HP ? no[B1_OFF + i] : no[B2_OFF + i - 2 * HP];
  const bool live = r < ncol;
  const int dst = pair_dst[first + min(r, ncol - 1)];
  // l-inf norm of the staged columns: eight threads per column take the
  // largest squared modulus over each pass's k range (components below N_u)
  const int mc = t >> 3, mj = t & 7;
  float m2 = 0.f, s = 0.f, inv_s = 0.f;
  __syncthreads();

  // layer 1: A row = hidden unit m of part (0: real, 1: imaginary); lane
  // half h multiplies the real (h = 0) or imaginary (h = 1) inputs. Row
  // block rb = wave (2 HB <= 4 blocks, so at most one per wavefront).
  {
    constexpr int NB = 2 * HB, PER1 = (NB + 3) / 4;
    static_assert(PER1 == 1, "one layer-1 row block per wavefront");
    floatx16 acc[PER1];
    const floatx4* arow[PER1];
#pragma unroll
    for (int i = 0; i < PER1; ++i) {
      const int rb = min(wave + 4 * i, NB - 1);
      arow[i] = reinterpret_cast<const floatx4*>(no) + (size_t)rb * (KH / 4) * 64 + lane;
      acc[i] = floatx16{};
    }
#pragma unroll
    for (int pass = 0; pass < PASSES; ++pass) {
      if (pass > 0) {
        __syncthreads();  // every wavefront is done with the previous pass
        stager.stage(xs4, Pr, ncol, pass);
        __syncthreads();
      }
      const floatx4* ap[PER1];
#pragma unroll
      for (int i = 0; i < PER1; ++i) ap[i] = arow[i] + pass * (KP / 4) * 64;
      if (wave < NB)  // wave-uniform
        rowblock_pipelined<KP / 4, 3>(acc[0], ap[0],
                                      reinterpret_cast<const floatx4*>(xs + r * XP + h * KP));
#pragma unroll
      for (int u = mj; u < KP; u += 8) {
        if (pass * KP + u < NU) {
          const float re = xs[mc * XP + u], im = xs[mc * XP + KP + u];
          m2 = fmaxf(m2, fmaf(re, re, im * im));
        }
      }
    }
    m2 = fmaxf(m2, __shfl_xor(m2, 4, 64));
    m2 = fmaxf(m2, __shfl_xor(m2, 2, 64));
    m2 = fmaxf(m2, __shfl_xor(m2, 1, 64));
    if (mj == 0) col_scale[mc] = sqrtf(m2);
    __syncthreads();  // every wavefront is done with the staged vectors
    s = col_scale[r];
    inv_s = s > 0.f ? 1.f / s : 0.f;
#pragma unroll
    for (int i = 0; i < PER1; ++i) {
      const int rb = wave + 4 * i;
      if (rb >= NB) continue;
      const int hpart = rb / HB, m0 = (rb % HB) * 32;
      const float* b1 = bias + hpart * HP + m0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        floatx4 v;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int row = 8 * q + 4 * h + jj;
          const float z = fmaf(acc[i][4 * q + jj], inv_s, b1[row]);
          v[jj] = (m0 + row < hidden) ? fmaxf(z, 0.f) : 0.f;
        }
        *reinterpret_cast<floatx4*>(hs + r * HPT + rb * 32 + 8 * q + 4 * h) = v;
      }
    }
  }
  __syncthreads();

  // layer 2: A row = output row of [Er | Ei]; row blocks ob = wave + 4 i
  float* prow = part + ((int64_t)rhs * n_pairs + dst) * PSTR;
  {
    constexpr int PER = (OB + 3) / 4;
    floatx16 acc[PER];
    const floatx4* arow[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int ob = min(wave + 4 * i, OB - 1);
      arow[i] = reinterpret_cast<const floatx4*>(no + W2_OFF) + (size_t)ob * (HP / 4) * 64 + lane;
      acc[i] = floatx16{};
    }
    // hidden units past the network's width are zero in the hidden tile and
    // in W2: the k loop stops at the last group holding a unit
    rowblock_products<PER, HP / 4, 2>(acc, arow,
                                   reinterpret_cast<const floatx4*>(hs + r * HPT + h * HP),
                                   (hidden + 3) / 4);
    if (live) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int ob = wave + 4 * i;
        if (ob >= OB) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r0 = ob * 32 + 8 * q + 4 * h;  // first of this lane's 4 rows
          if (r0 < 2 * NU) {
            floatx4 v;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const int orow = r0 + jj;
              const float b = orow < NU ? bias[2 * HP + orow]
                                        : (orow < 2 * NU ? bias[2 * HP + KH + orow - NU] : 0.f);
              v[jj] = s * (acc[i][4 * q + jj] + b);
            }
            *reinterpret_cast<floatx4*>(prow + r0) = v;
          }
        }
      }
    }
  }
}

// Operator-table product E = G_w P for box sizes whose columns do not fit
// in registers (N_u = 192): the scheme of the network kernel's first layer
// with M = K = 2 N_u, A read from the FP32 table in fragment order (per
// offset: 2 N_u / 32 row blocks of [[Gr, -Gi], [Gi, Gr]], KH/4 groups, 64
// lanes x 4 floats) and B from the box vectors staged in two passes.
template <int NU>
__global__ __launch_bounds__(kBlock, 4) void translate_staged_kernel(
    const float* __restrict__ table, const int32_t* __restrict__ items,
    const int32_t* __restrict__ pair_src, const int32_t* __restrict__ pair_dst,
    const float* __restrict__ P, float* __restrict__ part, int64_t n_box, int64_t n_pairs,
    int n_items) {
  constexpr int KH = (NU + 3) & ~3;
  constexpr int PASSES = staging_passes(KH);
  constexpr int KP = KH / PASSES;
  constexpr int XP = 2 * KP + 4;
  constexpr int OB = (2 * NU + 31) / 32;
  constexpr int PSTR = 2 * KH;
  __shared__ floatx4 xs4[32 * XP / 4];
  const float* xs = reinterpret_cast<const float*>(xs4);

  int o, first, ncol;
  if (!load_item(items, n_items, o, first, ncol)) return;  // grid padding
  const int rhs = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const float* Pr = P + (int64_t)rhs * n_box * 2 * KH;
  const ColumnStager<KH, XP, PASSES> stager(pair_src, first, ncol);
  stager.stage(xs4, Pr, ncol, 0);
  const bool live = r < ncol;
  const int dst = pair_dst[first + min(r, ncol - 1)];
  __syncthreads();
  const floatx4* Go = reinterpret_cast<const floatx4*>(table) + (size_t)o * OB * (KH / 4) * 64;
  float* prow = part + ((int64_t)rhs * n_pairs + dst) * PSTR;
  constexpr int PER = (OB + 3) / 4;
  floatx16 acc[PER];
  const floatx4* arow[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    arow[i] = Go + (size_t)min(wave + 4 * i, OB - 1) * (KH / 4) * 64 + lane;
    acc[i] = floatx16{};
  }
#pragma unroll
  for (int pass = 0; pass < PASSES; ++pass) {
    if (pass > 0) {
      __syncthreads();  // every wavefront is done with the previous pass
      stager.stage(xs4, Pr, ncol, pass);
      __syncthreads();
    }
    const floatx4* ap[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) ap[i] = arow[i] + pass * (KP / 4) * 64;
    rowblock_products<PER, KP / 4, 1>(acc, ap, reinterpret_cast<const floatx4*>(xs + r * XP + h * KP));
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int ob = wave + 4 * i;
      if (ob >= OB) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r0 = ob * 32 + 8 * q + 4 * h;
        if (r0 < 2 * NU)
          *reinterpret_cast<floatx4*>(prow + r0) =
              floatx4{acc[i][4 * q], acc[i][4 * q + 1], acc[i][4 * q + 2], acc[i][4 * q + 3]};
      }
    }
  }
}

// 16-bit matrix-core product on 8 values per lane (FP32 accumulation).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned uintx4 __attribute__((ext_vector_type(4)));
template <bool F16>
__device__ inline floatx16 mfma16(uintx4 a, uintx4 b, floatx16 c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a),
                                                 __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// The split-precision operator-table product for box sizes whose 16-bit
// columns do not fit in registers (N_u = 192, the paper's 4x4x4 dipoles),
// on v_mfma_f32_32x32x16_f16 / _bf16: the same products as the register
// kernels (G_h P_h + G_h P_l + G_l P_h, or G_h P_h alone), one workgroup per
// work item (up to 32 pairs of one offset). The item's 16-bit box vectors
// (stage 1's layout: per k-step of 8 coefficients, [re.hi | im.hi | re.lo |
// im.lo]) are staged whole in LDS, one column per row with a 16-byte pad so
// that the 32 columns' reads spread over the banks; wavefront w computes the
// 32-row blocks w, w + 4, w + 8 of [[Gr, -Gi], [Gi, Gr]] (M = K = 2 N_u),
// with the A values read from the operator image in matrix-core fragment
// order (per block, k-step and part: 64 lanes x 16 bytes contiguous). FP16:
// each result is multiplied by its offset's and its source box's scales
// (powers of two).
template <int NU, bool F16, int NPROD>
__global__ __launch_bounds__(kBlock, 2) void translate_staged_split_kernel(
    const unsigned short* __restrict__ table, const int32_t* __restrict__ items,
    const int32_t* __restrict__ pair_src, const int32_t* __restrict__ pair_dst,
    const float* __restrict__ P, float* __restrict__ part, int64_t n_box, int64_t n_pairs,
    int n_items, const float* __restrict__ off_scale, const float* __restrict__ box_scale) {
  constexpr int KH = (NU + 3) & ~3;
  constexpr int KHB = (NU + 7) & ~7;
  constexpr int NGB = KHB / 8;            // k-steps per half
  constexpr int VU = NGB * 4;             // 16-byte units per box vector
  constexpr int CPU = VU + 1;             // LDS pitch per column (units)
  constexpr int OB = (2 * NU + 31) / 32;  // 32-row blocks
  constexpr int PER = (OB + 3) / 4;       // blocks per wavefront
  constexpr int NPART = NPROD == 3 ? 2 : 1;
  constexpr int PSTR = 2 * KH;
  __shared__ uintx4 cols[32 * CPU];

  int o, first, ncol;
  if (!load_item(items, n_items, o, first, ncol)) return;  // grid padding
  const int rhs = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const uintx4* Pv = reinterpret_cast<const uintx4*>(P) + (int64_t)rhs * n_box * VU;
  // stage the item's columns (past ncol: the last pair again)
  for (int u = threadIdx.x; u < 32 * VU; u += kBlock) {
    const int c = u / VU, q = u - c * VU;
    const int src = pair_src[first + min(c, ncol - 1)];
    cols[c * CPU + q] = Pv[(int64_t)src * VU + q];
  }
  const int src_r = pair_src[first + min(r, ncol - 1)];
  const int dst = pair_dst[first + min(r, ncol - 1)];
  const float sc = F16 ? off_scale[o] * box_scale[(int64_t)rhs * n_box + src_r] : 1.f;
  __syncthreads();

  const uintx4* Ao = reinterpret_cast<const uintx4*>(table) + (size_t)o * OB * NGB * NPART * 64;
  const uintx4* arow[PER];
  floatx16 acc[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    arow[i] = Ao + (size_t)min(wave + 4 * i, OB - 1) * NGB * NPART * 64 + lane;
    acc[i] = floatx16{};
  }
  const uintx4* col = cols + r * CPU;
#pragma unroll 4
  for (int g = 0; g < NGB; ++g) {
    const uintx4 bh = col[4 * g + h];
    const uintx4 bl = NPROD == 3 ? col[4 * g + 2 + h] : uintx4{};
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uintx4 ah = arow[i][(g * NPART) * 64];
      acc[i] = mfma16<F16>(ah, bh, acc[i]);
      if (NPROD == 3) {
        const uintx4 al = arow[i][(g * NPART + 1) * 64];
        acc[i] = mfma16<F16>(ah, bl, acc[i]);
        acc[i] = mfma16<F16>(al, bh, acc[i]);
      }
    }
  }
  if (r < ncol) {
    float* prow = part + ((int64_t)rhs * n_pairs + dst) * PSTR;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int ob = wave + 4 * i;
      if (ob >= OB) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r0 = ob * 32 + 8 * q + 4 * h;
        if (r0 < 2 * NU)
          *reinterpret_cast<floatx4*>(prow + r0) =
              floatx4{acc[i][4 * q], acc[i][4 * q + 1], acc[i][4 * q + 2], acc[i][4 * q + 3]} *
              sc;
      }
    }
  }
}

int grid_for(int64_t total) {
  const int64_t g = (total + kBlock - 1) / kBlock;
  return (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

}  // namespace

bool network_shape_supported(int nu, int hidden) {
  return (nu == 24 || nu == 81 || nu == 192) && hidden >= 1 && hidden <= kMaxHidden;
}

int network_hp(int hidden) { return hidden <= 32 ? 32 : 64; }

size_t network_image_bytes(const Plan& p, int hidden) {
  return (size_t)std::max<int32_t>(p.n_off(), 1) *
         (size_t)image_floats(p.nu, p.kh, network_hp(hidden)) * sizeof(float);
}

int launch_network_pack(const Plan& p, int hidden, const void* W1, const void* b1,
                        const void* W2, const void* b2, float* img, void* stream) {
  const int hp = network_hp(hidden);
  const int64_t total = (int64_t)p.n_off() * image_floats(p.nu, p.kh, hp);
  if (total == 0) return 0;
  hipLaunchKernelGGL(network_pack_kernel, dim3(grid_for(total)), dim3(kBlock), 0,
                     (hipStream_t)stream, (const float2*)W1, (const float2*)b1,
                     (const float2*)W2, (const float2*)b2, img, (int64_t)p.n_off(), p.nu,
                     p.kh, hp, hidden);
  return (int)hipGetLastError();
}

// Launch with timing events when the stage has them (plain launch otherwise,
// as under graph capture).
#define UBF_LAUNCH(T0, T1, KERNEL, GRID, STREAM, ...)                                     \
  do {                                                                                   \
    if ((T0) || (T1))                                                                    \
      hipExtLaunchKernelGGL(KERNEL, GRID, dim3(kBlock), 0, STREAM, T0, T1, 0, __VA_ARGS__); \
    else                                                                                 \
      hipLaunchKernelGGL(KERNEL, GRID, dim3(kBlock), 0, STREAM, __VA_ARGS__);            \
  } while (0)

int launch_translate_cvfcnn(const Plan& p, const float* P, float* part, int nrhs, void* stream,
                            const StageEvents* ev) {
  hipStream_t s = (hipStream_t)stream;
  const int nit = (int)p.n_items();
  hipEvent_t t0 = ev ? ev->start : nullptr, t1 = ev ? ev->stop : nullptr;
  if (nit == 0) {
    if (ev) {
      hipError_t e = hipEventRecord(t0, s);
      if (e == hipSuccess) e = hipEventRecord(t1, s);
      return (int)e;
    }
    return 0;
  }
  const dim3 grid((unsigned)((nit + 7) / 8 * 8), nrhs);
#define UBF_NET(NU, HB)                                                                    \
  UBF_LAUNCH(t0, t1, (translate_cvfcnn_kernel<NU, HB>), grid, s, p.d_net, p.d_items,       \
             p.d_pair_src, p.d_pair_dst, P, part, p.n_box, p.n_pairs(), p.hidden, nit)
  const bool wide = p.hidden > 32;
  switch (p.nu) {
    case 24: if (wide) UBF_NET(24, 2); else UBF_NET(24, 1); break;
    case 81: if (wide) UBF_NET(81, 2); else UBF_NET(81, 1); break;
    case 192: if (wide) UBF_NET(192, 2); else UBF_NET(192, 1); break;
    default: return (int)hipErrorInvalidValue;  // rejected when the networks are set
  }
#undef UBF_NET
  return (int)hipGetLastError();
}

bool staged_translate_supported(const Plan& p) { return p.nu == 192; }

int launch_translate_staged(const Plan& p, const float* P, float* part, int nrhs, void* stream,
                            const StageEvents* ev) {
  hipStream_t s = (hipStream_t)stream;
  const int nit = (int)p.n_items();
  hipEvent_t t0 = ev ? ev->start : nullptr, t1 = ev ? ev->stop : nullptr;
  if (nit == 0) {
    if (ev) {
      hipError_t e = hipEventRecord(t0, s);
      if (e == hipSuccess) e = hipEventRecord(t1, s);
      return (int)e;
    }
    return 0;
  }
  if (p.nu != 192) return (int)hipErrorInvalidValue;
  const dim3 grid((unsigned)((nit + 7) / 8 * 8), nrhs);
  if (!p.split()) {
    UBF_LAUNCH(t0, t1, translate_staged_kernel<192>, grid, s, p.d_table, p.d_items,
               p.d_pair_src, p.d_pair_dst, P, part, p.n_box, p.n_pairs(), nit);
    return (int)hipGetLastError();
  }
  const unsigned short* tb = reinterpret_cast<const unsigned short*>(p.d_table);
#define UBF_STAGED16(F16, NPROD)                                                             \
  UBF_LAUNCH(t0, t1, (translate_staged_split_kernel<192, F16, NPROD>), grid, s, tb, p.d_items, \
             p.d_pair_src, p.d_pair_dst, P, part, p.n_box, p.n_pairs(), nit, p.d_off_scale,    \
             p.d_box_scale)
  if (p.precision == 1) UBF_STAGED16(false, 3);
  else if (p.precision == 2) UBF_STAGED16(true, 3);
  else UBF_STAGED16(true, 1);
#undef UBF_STAGED16
  return (int)hipGetLastError();
}
#undef UBF_LAUNCH

}  // namespace ubf

// Host-side plan of the far-zone product: geometry, far set, work
// partition and the operator table image. Everything here runs on the CPU
// at plan creation; nothing touches a device.
#pragma once

#include <complex>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

namespace ubf {

// Columns (box pairs) per translation work unit: four wavefronts of 32.
constexpr int kChunk = 128;
// Translation workgroups: two resident per compute unit on 256 CUs.
constexpr int kTranslateGroups = 512;
// Stage-2 kernels of the 16-bit forms, chosen per plan (ubf_plan_tune or
// ubf_plan_schedule): persistent workgroups over chunks of 128 pairs, one
// right-hand side per grid row (kSplitChunks) or every right-hand side of a
// chunk in turn (kSplitChunksWalk, one operator staging for all of them);
// rounds of four 32-pair items per workgroup, two workgroups per compute
// unit with one operator buffer each (kSplitRounds) or one with two buffers
// and the next operator copied ahead (kSplitRoundsDouble). All give the
// same result bit for bit.
enum SplitKernel { kSplitChunks = 0, kSplitChunksWalk = 1, kSplitRounds = 2,
                   kSplitRoundsDouble = 3 };
// Default workgroups of the round kernels: two per compute unit.
constexpr int kRoundGroups = 512;
// Largest persistent grid the tuner may pick (workspace room for its
// chunk ranges is reserved at this size).
constexpr int kMaxTranslateGroups = 4096;

// Padded half-length of a planar box vector: N_u rounded up to a multiple
// of 4. A box vector is stored as [re(N_u), 0 pad | im(N_u), 0 pad], 2*kh
// floats, so both halves start 16-byte aligned.
inline int half_len(int nu) { return (nu + 3) & ~3; }

// Split-precision layouts (BF16 hi/lo): half-length rounded up to a
// multiple of 8 so a lane's 8 consecutive BF16 values are one 16-byte read.
inline int half_len_bf16(int nu) { return (nu + 7) & ~7; }

// Round-to-nearest-even FP32 -> FP16 bits (finite inputs within range).
inline uint16_t fp16_bits(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t sign = (x >> 16) & 0x8000u;
  const int32_t e = (int32_t)((x >> 23) & 0xFF) - 127;
  uint32_t m = x & 0x7FFFFFu;
  if (e > 15) return (uint16_t)(sign | 0x7C00u);          // overflow -> inf
  if (e >= -14) {                                          // normal
    uint32_t h = ((uint32_t)(e + 15) << 10) | (m >> 13);
    const uint32_t rest = m & 0x1FFFu;
    if (rest > 0x1000u || (rest == 0x1000u && (h & 1u))) ++h;  // may carry into exp
    return (uint16_t)(sign | h);
  }
  if (e < -25) return (uint16_t)sign;                      // underflow -> 0
  m |= 0x800000u;                                          // subnormal
  const int shift = -e - 14 + 13;                          // 14..24
  uint32_t h = m >> shift;
  const uint32_t rest = m & ((1u << shift) - 1u), half = 1u << (shift - 1);
  if (rest > half || (rest == half && (h & 1u))) ++h;
  return (uint16_t)(sign | h);
}
inline float fp16_value(uint16_t b) {
  const uint32_t sign = (uint32_t)(b & 0x8000u) << 16;
  const int e = (b >> 10) & 0x1F;
  const uint32_t m = b & 0x3FFu;
  float f;
  if (e == 0) {
    f = (float)m * 5.9604644775390625e-08f;  // 2^-24
  } else if (e == 31) {
    const uint32_t u = sign | 0x7F800000u | (m << 13);
    std::memcpy(&f, &u, 4);
    return f;
  } else {
    const uint32_t u = ((uint32_t)(e - 15 + 127) << 23) | (m << 13);
    std::memcpy(&f, &u, 4);
  }
  return sign ? -f : f;
}

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
inline uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
inline float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Free-space dyadic Green's function of Eq. (5)-(6), FP64, time
// convention exp(+j omega t): D(R) = psi(R) { I (1 - j/kR - 1/(kR)^2)
//   - Rhat Rhat (1 - 3j/kR - 3/(kR)^2) },  psi = -j k eta e^{-jkR}/(4 pi R).
void dyadic_green(const double R[3], double k, double eta,
                  std::complex<double> D[3][3]);

// Cell-centred site offsets from the box centre, site s = (mx*n_d+my)*n_d+mz.
std::vector<double> site_offsets(double a, int n_d);

// G_w in FP64, row-major n_u x n_u complex: entry ((l,alpha),(s,beta)) is
// D(a*w + r_l - r_s)[alpha][beta] (Eq. 12-13).
void operator_fp64(const int32_t w[3], double a, double k, double eta, int n_d,
                   std::vector<std::complex<double>>& G);

struct Plan {
  // Problem.
  int64_t n_box = 0;
  std::vector<int32_t> boxes;  // 3 * n_box
  // Independent scatterers: boxes [scat_ptr[s], scat_ptr[s+1]) form
  // scatterer s; far-zone pairs never join two scatterers.
  std::vector<int64_t> scat_ptr;
  double a = 0, k = 0, eta = 0;
  int n_d = 0, nu = 0, kh = 0, far_mode = 0, precision = 0;

  // Far set, grouped by offset (offset index ascending, then test box).
  std::vector<int32_t> offsets;    // 3 * n_off, lexicographic order
  std::vector<int64_t> off_ptr;    // n_off + 1
  std::vector<int32_t> pair_test;  // n_pairs
  std::vector<int32_t> pair_src;   // n_pairs
  std::vector<int32_t> pair_off;   // n_pairs
  std::vector<int32_t> test_ptr;   // n_box + 1: pairs of each test box ...
  std::vector<int32_t> test_pos;   // ... as positions in the grouped order
  std::vector<int32_t> pair_dst;   // grouped position -> test-major position
  std::vector<int32_t> chunks;     // 4 per chunk: offset, begin, count, 0
  // Work items of the kernels that stage box vectors in LDS: 4 per item of
  // up to 32 consecutive pairs of one offset: offset, first pair, count, 0.
  std::vector<int32_t> items;
  std::vector<int32_t> wg_ptr;     // chunk range of each translation workgroup
  // Rounds of the 16-bit translation (one workgroup of four wavefronts per
  // compute unit): each workgroup walks a contiguous range of items in
  // rounds; round k gives wavefront w the item (offset, first pair, count,
  // flags) at rounds[4 * (4 k + w)]; an empty slot has count 0. A round that
  // starts a run of one offset (a segment) has flags bit 0 set and carries
  // the offset of the workgroup's next segment plus one in bits 1.. (0: none).
  std::vector<int32_t> rounds;
  std::vector<int32_t> wg_round_ptr;  // round range of each workgroup
  // Stage-2 kernel of the 16-bit forms (enum SplitKernel).
  int split_kernel = kSplitChunks;
  // Operators evaluated by the translation kernel from the offsets (FP64
  // Green's function) instead of read from a table; the table is empty.
  bool gen_ops = false;
  int32_t n_orbits = 0;

  // Operator table image: per offset two planes (re, im) of nu rows of kh
  // floats; columns >= nu are zero. Split precision instead stores, per
  // offset, planes re.hi, im.hi, re.lo, im.lo (the hi half first) of nu rows
  // of khb 16-bit values.
  std::vector<float> table;
  std::vector<uint16_t> table_bf16;  // 16-bit image (BF16 or FP16 bits)
  // FP16 forms: operator o is stored divided by off_scale[o] (a power of
  // two), so that every operator fits the FP16 range.
  std::vector<float> off_scale;
  int khb = 0;
  // 16-bit forms (precision 1: BF16 hi/lo; 2: FP16 hi/lo; 3: FP16 single).
  bool split() const { return precision >= 1; }
  bool fp16() const { return precision >= 2; }
  int nprod() const { return precision == 3 ? 1 : 3; }

  int64_t n_pairs() const { return (int64_t)pair_src.size(); }
  int32_t n_off() const { return (int32_t)(offsets.size() / 3); }
  int64_t n_chunks() const { return (int64_t)(chunks.size() / 4); }
  int64_t n_items() const { return (int64_t)(items.size() / 4); }
  int32_t n_groups() const { return (int32_t)wg_ptr.size() - 1; }
  int32_t n_round_groups() const { return (int32_t)wg_round_ptr.size() - 1; }
  int32_t n_scat() const { return (int32_t)scat_ptr.size() - 1; }
  size_t plane_floats() const { return (size_t)nu * kh; }
  size_t op_floats() const { return 2 * plane_floats(); }
  // FP32 operators of boxes whose columns do not fit in registers
  // (N_u = 192) are stored in the matrix-core fragment order of the staged
  // kernel: per 32-row block of [[Gr, -Gi], [Gi, Gr]], per group of four
  // k-steps, 64 lanes x 4 floats.
  bool staged() const { return !split() && nu == 192; }
  size_t staged_op_floats() const { return (size_t)((2 * nu + 31) / 32) * (kh / 4) * 256; }
  // 16-bit operators of 192-coefficient boxes are stored in the fragment
  // order of the staged split kernel: per 32-row block, k-step of 8 and part
  // (hi, lo; hi only for the single-product form), 64 lanes x 8 values.
  bool staged_split() const { return split() && nu == 192; }
  size_t staged_split_halves() const {
    return (size_t)((2 * nu + 31) / 32) * (khb / 8) * (precision == 3 ? 1 : 2) * 64 * 8;
  }
  int pstride() const { return 2 * kh; }              // partial rows, floats
  // Box vectors of stage 1 -> 2, in floats: FP32 [re | im] halves, or in
  // split mode [re: hi, lo | im: hi, lo] BF16 runs of khb values.
  int vstride() const { return split() ? 2 * khb : 2 * kh; }
  size_t table_bytes() const {
    return split() ? table_bf16.size() * sizeof(uint16_t) : table.size() * sizeof(float);
  }

  // Binding.
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int32_t max_nrhs = 0;
  // Device pointers into the workspace.
  float* d_table = nullptr;
  int32_t* d_chunks = nullptr;
  int32_t* d_items = nullptr;
  int32_t* d_wg_ptr = nullptr;
  int32_t* d_rounds = nullptr;
  int32_t* d_wg_round_ptr = nullptr;
  int32_t* d_pair_src = nullptr;
  int32_t* d_test_ptr = nullptr;
  int32_t* d_pair_dst = nullptr;
  int64_t* d_nb_ptr = nullptr;
  float* d_P = nullptr;
  float* d_part = nullptr;
  float* d_off_scale = nullptr;  // [n_off] (FP16 forms)
  int32_t* d_offsets = nullptr;  // [n_off][3] integer offsets (generated operators)
  float* d_box_scale = nullptr;  // [max_nrhs][n_box] box-vector scales (FP16 forms)

  // Networks standing in for the operators (Sec. 3): hidden width (0 = none,
  // stage 2 uses the operator table) and the device image, owned by the caller.
  int hidden = 0;
  const float* d_net = nullptr;

  // Basis.
  bool has_basis = false;
  std::vector<int64_t> nb_ptr;  // n_box + 1
  const void* d_S = nullptr;
  const void* d_T = nullptr;
  int64_t nb_total() const {
    return has_basis ? nb_ptr.back() : n_box * (int64_t)nu;
  }
};

// Workspace layout, in bytes from the workspace start.
struct Layout {
  size_t table, chunks, items, wg_ptr, rounds, wg_round_ptr, pair_src, pair_dst, test_ptr, nb_ptr,
      P, part, off_scale, box_scale, offsets, total;
};
Layout workspace_layout(const Plan& p, int32_t max_nrhs);

// The per-call intermediates of one product of nrhs right-hand sides (box
// vectors, partial rows with their spare row, FP16 box scales), laid out
// from offset 0 of a scratch region, in bytes.
struct ScratchLayout {
  size_t P, part, box_scale, total;
};
ScratchLayout scratch_layout(const Plan& p, int32_t nrhs);

// Validate and build; returns an empty string on success, else the reason.
// scat_ptr (n_scat + 1 prefix offsets into the boxes) splits the boxes into
// independent scatterers; NULL means one scatterer. operators: 0 = table
// built here, 1 = evaluated by the translation kernel (16-bit forms, n_d
// 1..3; no table).
std::string build_plan(const int32_t* box_ijk, int64_t n_box, double a,
                       double k, double eta, int n_d, int far_mode,
                       int precision, int operators, const int64_t* scat_ptr,
                       int64_t n_scat, Plan& out);

// Rounds of the 16-bit translation for `groups` workgroups (rounded up to a
// multiple of 8, at most kMaxTranslateGroups, at most one per item), each
// taking a contiguous range of items balanced by count; rewrites p.rounds
// and p.wg_round_ptr.
void build_rounds(Plan& p, int64_t groups);
// Upper bound of the round count over every group count build_rounds takes.
int64_t max_rounds(const Plan& p);

// Contiguous chunk ranges for `groups` persistent translation workgroups
// (rounded up to a multiple of 8, at most kMaxTranslateGroups), balanced by
// chunk count; rewrites p.wg_ptr.
void partition_groups(Plan& p, int64_t groups);

}  // namespace ubf

// Host plan builder: validation, far set (Algorithm 2), offset grouping,
// symmetry orbits (Sec. 2.2) and the FP32 operator table (Eq. 5-6, 13).
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <thread>
#include <numeric>
#include <unordered_map>

namespace ubf {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEta0 = 376.730313668;
// Dense box-index grids above this many cells use a hash map instead.
constexpr int64_t kDenseCells = int64_t(1) << 24;
// Largest operator table accepted (bytes).
constexpr double kMaxTableBytes = 16.0 * (1ull << 30);

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Lookup of a box index from integer coordinates. Small bounding grids use
// a dense array; larger ones a hash map keyed on the exact coordinate
// triple (any int32 >= 0 per axis), so distinct boxes never share a key.
struct BoxIndex {
  struct Key {
    int32_t x, y, z;
    bool operator==(const Key& o) const { return x == o.x && y == o.y && z == o.z; }
  };
  struct KeyHash {
    size_t operator()(const Key& k) const {
      uint64_t h = (uint32_t)k.x;
      h = h * 0x9E3779B97F4A7C15ull ^ (uint32_t)k.y;
      h = h * 0x9E3779B97F4A7C15ull ^ (uint32_t)k.z;
      return (size_t)(h ^ (h >> 31));
    }
  };
  int64_t nx = 0, ny = 0, nz = 0;
  std::vector<int32_t> dense;
  std::unordered_map<Key, int32_t, KeyHash> sparse;
  bool use_dense = true;

  // Index boxes b[0..n) (3 coordinates each, all >= 0); false on a duplicate.
  bool build(const int32_t* b, int64_t n) {
    int64_t mx = 0, my = 0, mz = 0;
    for (int64_t i = 0; i < n; ++i) {
      mx = std::max<int64_t>(mx, b[3 * i]);
      my = std::max<int64_t>(my, b[3 * i + 1]);
      mz = std::max<int64_t>(mz, b[3 * i + 2]);
    }
    nx = mx + 1;
    ny = my + 1;
    nz = mz + 1;
    // the product of three extents up to 2^31 overflows int64: test stepwise
    use_dense = nx <= kDenseCells && ny <= kDenseCells && nz <= kDenseCells &&
                nx * ny <= kDenseCells && nx * ny * nz <= kDenseCells;
    dense.clear();
    sparse.clear();
    if (use_dense) {
      dense.assign((size_t)(nx * ny * nz), -1);
      for (int64_t i = 0; i < n; ++i) {
        int32_t& slot = dense[((size_t)b[3 * i] * ny + b[3 * i + 1]) * nz + b[3 * i + 2]];
        if (slot >= 0) return false;
        slot = (int32_t)i;
      }
    } else {
      sparse.reserve((size_t)n * 2);
      for (int64_t i = 0; i < n; ++i)
        if (!sparse.emplace(Key{b[3 * i], b[3 * i + 1], b[3 * i + 2]}, (int32_t)i).second)
          return false;
    }
    return true;
  }
  int32_t find(int64_t x, int64_t y, int64_t z) const {
    if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return -1;
    if (use_dense) return dense[((size_t)x * ny + y) * nz + z];
    auto it = sparse.find(Key{(int32_t)x, (int32_t)y, (int32_t)z});
    return it == sparse.end() ? -1 : it->second;
  }
};

int32_t cheb(int64_t x, int64_t y, int64_t z) {
  return (int32_t)std::max({std::llabs(x), std::llabs(y), std::llabs(z)});
}

int64_t floordiv2(int64_t c) { return c >= 0 ? c / 2 : -((-c + 1) / 2); }

// One offset's operator image in the table layout. FP32: planes re, im of
// nu rows of kh floats. Split: G is rounded to FP32 first (as in the FP32
// path), then hi = bf16(G), lo = bf16(G - hi); planes re.hi, im.hi, re.lo,
// im.lo of nu rows of khb values. Padding columns are zero.
// The 16-bit image of 192-coefficient boxes, in the matrix-core fragment
// order of the staged split kernel: per 32-row block b of the real form
// [[Gr, -Gi], [Gi, Gr]], k-step g (8 values of each K half) and part (hi,
// then lo unless the single-product form), 64 lanes x 8 values: lane l holds
// row 32 b + l % 32 and K half l / 32 (the real inputs for 0, the imaginary
// ones for 1), values k = 8 g .. 8 g + 7. Each operator value v (divided by
// the offset's power-of-two scale in the FP16 forms) is hi = round16(v),
// lo = round16(v - hi), as in the plane layout.
void staged_split_image(const Plan& P, const std::vector<std::complex<double>>& G, double inv,
                        uint16_t* out) {
  const int nb = (2 * P.nu + 31) / 32, ng = P.khb / 8, np = P.precision == 3 ? 1 : 2;
  for (int b = 0; b < nb; ++b)
    for (int g = 0; g < ng; ++g)
      for (int q = 0; q < np; ++q)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 8; ++j) {
            const int row = 32 * b + (l & 31), h = l >> 5, k = 8 * g + j;
            double v = 0.0;
            if (row < 2 * P.nu && k < P.nu) {
              const bool ei = row >= P.nu;
              const std::complex<double> c = G[(size_t)(ei ? row - P.nu : row) * P.nu + k];
              v = !ei ? (h == 0 ? c.real() : -c.imag()) : (h == 0 ? c.imag() : c.real());
            }
            const float f = (float)(v * inv);
            uint16_t bits;
            if (P.fp16()) {
              const uint16_t hi = fp16_bits(f);
              bits = q == 0 ? hi : fp16_bits(f - fp16_value(hi));
            } else {
              const uint16_t hi = bf16_bits(f);
              bits = q == 0 ? hi : bf16_bits(f - bf16_value(hi));
            }
            out[((((size_t)b * ng + g) * np + q) * 64 + l) * 8 + j] = bits;
          }
}

void offset_image(const Plan& P, const int32_t* w, std::vector<std::complex<double>>& G,
                  char* dst, float* scale) {
  operator_fp64(w, P.a, P.k, P.eta, P.n_d, G);
  *scale = 1.0f;
  if (P.staged_split()) {
    double inv = 1.0;
    if (P.fp16()) {  // power of two bringing the largest |Re|, |Im| to [2^14, 2^15)
      double mx = 0.0;
      for (const auto& g : G) mx = std::max({mx, std::abs(g.real()), std::abs(g.imag())});
      const int e = mx > 0.0 ? std::ilogb(mx) - 14 : 0;
      *scale = (float)std::ldexp(1.0, e);
      inv = std::ldexp(1.0, -e);  // exact power of two
    }
    staged_split_image(P, G, inv, (uint16_t*)dst);
    return;
  }
  if (P.fp16()) {
    // power of two bringing the largest |Re|, |Im| to [2^14, 2^15)
    double mx = 0.0;
    for (const auto& g : G) mx = std::max({mx, std::abs(g.real()), std::abs(g.imag())});
    const int e = mx > 0.0 ? std::ilogb(mx) - 14 : 0;
    *scale = (float)std::ldexp(1.0, e);
    const double inv = std::ldexp(1.0, -e);  // exact power of two
    const uint16_t zero = 0;
    const size_t plane = (size_t)P.nu * P.khb;
    uint16_t* base = (uint16_t*)dst;
    std::fill(base, base + 4 * plane, zero);
    for (int u = 0; u < P.nu; ++u)
      for (int v = 0; v < P.nu; ++v) {
        const std::complex<double> g = G[(size_t)u * P.nu + v];
        const float parts[2] = {(float)(g.real() * inv), (float)(g.imag() * inv)};
        for (int c = 0; c < 2; ++c) {
          const uint16_t hi = fp16_bits(parts[c]);
          const uint16_t lo = fp16_bits(parts[c] - fp16_value(hi));
          base[c * plane + (size_t)u * P.khb + v] = hi;
          base[(2 + c) * plane + (size_t)u * P.khb + v] = lo;
        }
      }
    return;
  }
  if (P.staged()) {
    // block b, group g, lane l (row r = l % 32 of the block, K half h = l / 32:
    // the real inputs for h = 0, the imaginary ones for h = 1), k-steps
    // 4g..4g+3: Er rows take (Gr, -Gi), Ei rows (Gi, Gr); rows past 2 N_u and
    // columns past N_u are zero
    const int g4 = P.kh / 4, nb = (2 * P.nu + 31) / 32;
    float* f = (float*)dst;
    for (int b = 0; b < nb; ++b)
      for (int g = 0; g < g4; ++g)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 4; ++j) {
            const int row = 32 * b + (l & 31), h = l >> 5, k = 4 * g + j;
            double v = 0.0;
            if (row < 2 * P.nu && k < P.nu) {
              const bool ei = row >= P.nu;
              const std::complex<double> c = G[(size_t)(ei ? row - P.nu : row) * P.nu + k];
              v = !ei ? (h == 0 ? c.real() : -c.imag()) : (h == 0 ? c.imag() : c.real());
            }
            f[(((size_t)b * g4 + g) * 64 + l) * 4 + j] = (float)v;
          }
    return;
  }
  if (!P.split()) {
    const size_t plane = P.plane_floats();
    float* re = (float*)dst;
    float* im = re + plane;
    std::fill(re, re + 2 * plane, 0.0f);
    for (int u = 0; u < P.nu; ++u)
      for (int v = 0; v < P.nu; ++v) {
        re[(size_t)u * P.kh + v] = (float)G[(size_t)u * P.nu + v].real();
        im[(size_t)u * P.kh + v] = (float)G[(size_t)u * P.nu + v].imag();
      }
  } else {
    const size_t plane = (size_t)P.nu * P.khb;
    uint16_t* base = (uint16_t*)dst;
    std::fill(base, base + 4 * plane, (uint16_t)0);
    for (int u = 0; u < P.nu; ++u)
      for (int v = 0; v < P.nu; ++v) {
        const std::complex<double> g = G[(size_t)u * P.nu + v];
        const float parts[2] = {(float)g.real(), (float)g.imag()};
        for (int c = 0; c < 2; ++c) {
          const uint16_t hi = bf16_bits(parts[c]);
          const uint16_t lo = bf16_bits(parts[c] - bf16_value(hi));
          base[c * plane + (size_t)u * P.khb + v] = hi;
          base[(2 + c) * plane + (size_t)u * P.khb + v] = lo;
        }
      }
  }
}

// Process-wide cache of operator images for offsets within +-3 (every
// ILIST offset), keyed by the exact parameters; bounded in bytes. Plans of
// repeated problems (serving) then skip the FP64 Green's evaluations.
struct ImageKey {
  double a, k, eta;
  int32_t n_d, precision, w0, w1, w2;
  bool operator==(const ImageKey& o) const {
    return a == o.a && k == o.k && eta == o.eta && n_d == o.n_d &&
           precision == o.precision && w0 == o.w0 && w1 == o.w1 && w2 == o.w2;
  }
};
struct ImageKeyHash {
  size_t operator()(const ImageKey& x) const {
    uint64_t h = 0;
    auto mix = [&h](uint64_t v) { h = (h ^ v) * 0x100000001B3ull + 0x9E3779B97F4A7C15ull; };
    uint64_t bits;
    std::memcpy(&bits, &x.a, 8); mix(bits);
    std::memcpy(&bits, &x.k, 8); mix(bits);
    std::memcpy(&bits, &x.eta, 8); mix(bits);
    mix((uint32_t)x.n_d); mix((uint32_t)x.precision);
    mix((uint32_t)x.w0); mix((uint32_t)x.w1); mix((uint32_t)x.w2);
    return (size_t)h;
  }
};
constexpr size_t kImageCacheBytes = size_t(256) << 20;
std::mutex g_image_mu;
std::unordered_map<ImageKey, std::vector<char>, ImageKeyHash> g_images;
size_t g_image_bytes = 0;

bool cacheable(const int32_t* w) {
  return std::abs(w[0]) <= 3 && std::abs(w[1]) <= 3 && std::abs(w[2]) <= 3;
}
ImageKey image_key(const Plan& P, const int32_t* w) {
  return ImageKey{P.a, P.k, P.eta, P.n_d, P.precision, w[0], w[1], w[2]};
}
// An entry holds the image followed by its float scale.
bool image_cache_get(const Plan& P, const int32_t* w, char* dst, size_t bytes, float* scale) {
  if (!cacheable(w)) return false;
  std::lock_guard<std::mutex> lock(g_image_mu);
  auto it = g_images.find(image_key(P, w));
  if (it == g_images.end() || it->second.size() != bytes + sizeof(float)) return false;
  std::memcpy(dst, it->second.data(), bytes);
  std::memcpy(scale, it->second.data() + bytes, sizeof(float));
  return true;
}
void image_cache_put(const Plan& P, const int32_t* w, const char* src, size_t bytes,
                     float scale) {
  if (!cacheable(w)) return;
  std::lock_guard<std::mutex> lock(g_image_mu);
  if (g_image_bytes + bytes > kImageCacheBytes) return;
  std::vector<char> entry(src, src + bytes);
  entry.resize(bytes + sizeof(float));
  std::memcpy(entry.data() + bytes, &scale, sizeof(float));
  auto ins = g_images.emplace(image_key(P, w), std::move(entry));
  if (ins.second) g_image_bytes += bytes;
}

}  // namespace

void dyadic_green(const double R[3], double k, double eta,
                  std::complex<double> D[3][3]) {
  const double r = std::sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
  const double rh[3] = {R[0] / r, R[1] / r, R[2] / r};
  const double kr = k * r;
  const std::complex<double> j(0.0, 1.0);
  const std::complex<double> psi =
      -j * k * eta * std::exp(-j * kr) / (4.0 * kPi * r);
  const std::complex<double> c_iso = 1.0 - j / kr - 1.0 / (kr * kr);
  const std::complex<double> c_rr = 1.0 - 3.0 * j / kr - 3.0 / (kr * kr);
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q)
      D[p][q] = psi * ((p == q ? c_iso : 0.0) - rh[p] * rh[q] * c_rr);
}

std::vector<double> site_offsets(double a, int n_d) {
  std::vector<double> r;
  r.reserve(3 * n_d * n_d * n_d);
  for (int mx = 0; mx < n_d; ++mx)
    for (int my = 0; my < n_d; ++my)
      for (int mz = 0; mz < n_d; ++mz) {
        r.push_back(a * ((mx + 0.5) / n_d - 0.5));
        r.push_back(a * ((my + 0.5) / n_d - 0.5));
        r.push_back(a * ((mz + 0.5) / n_d - 0.5));
      }
  return r;
}

void operator_fp64(const int32_t w[3], double a, double k, double eta, int n_d,
                   std::vector<std::complex<double>>& G) {
  // The sites form one uniform lattice of step a / n_d, so r_l - r_s depends
  // only on the lattice difference d = m_l - m_s in [-(n_d-1), n_d-1]^3:
  // evaluate D once per difference, then fill the site-pair blocks.
  const int nd3 = n_d * n_d * n_d, nu = 3 * nd3;
  const int span = 2 * n_d - 1;
  const double step = a / n_d;
  std::vector<std::complex<double>> Dd((size_t)span * span * span * 9);
  for (int dx = 0; dx < span; ++dx)
    for (int dy = 0; dy < span; ++dy)
      for (int dz = 0; dz < span; ++dz) {
        const double R[3] = {a * w[0] + step * (dx - (n_d - 1)),
                             a * w[1] + step * (dy - (n_d - 1)),
                             a * w[2] + step * (dz - (n_d - 1))};
        std::complex<double> D[3][3];
        dyadic_green(R, k, eta, D);
        std::complex<double>* out = &Dd[(((size_t)dx * span + dy) * span + dz) * 9];
        for (int al = 0; al < 3; ++al)
          for (int be = 0; be < 3; ++be) out[3 * al + be] = D[al][be];
      }
  G.assign((size_t)nu * nu, 0.0);
  for (int l = 0; l < nd3; ++l) {
    const int lx = l / (n_d * n_d), ly = (l / n_d) % n_d, lz = l % n_d;
    for (int s = 0; s < nd3; ++s) {
      const int sx = s / (n_d * n_d), sy = (s / n_d) % n_d, sz = s % n_d;
      const std::complex<double>* D =
          &Dd[((((size_t)(lx - sx + n_d - 1)) * span + (ly - sy + n_d - 1)) * span +
               (lz - sz + n_d - 1)) * 9];
      for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be)
          G[(size_t)(3 * l + al) * nu + 3 * s + be] = D[3 * al + be];
    }
  }
}

// The four wavefronts of a group work on one chunk at a time, so a group's
// time is its number of chunks whatever their fill: ranges are balanced by
// chunk count. Trailing groups may get empty ranges.
void partition_groups(Plan& P, int64_t groups) {
  const int64_t nch = P.n_chunks();
  groups = std::min<int64_t>(groups, std::max<int64_t>(nch, 1));
  groups = std::min<int64_t>((groups + 7) / 8 * 8, kMaxTranslateGroups);
  P.wg_ptr.assign(groups + 1, (int32_t)nch);
  P.wg_ptr[0] = 0;
  for (int64_t g = 1; g < groups; ++g) P.wg_ptr[g] = (int32_t)((nch * g + groups - 1) / groups);
}

void build_rounds(Plan& P, int64_t groups) {
  const int64_t ni = P.n_items();
  groups = std::min<int64_t>(groups, std::max<int64_t>(ni, 1));
  groups = std::min<int64_t>((groups + 7) / 8 * 8, kMaxTranslateGroups);
  P.rounds.clear();
  P.wg_round_ptr.assign(groups + 1, 0);
  const int32_t* it = P.items.data();
  for (int64_t g = 0; g < groups; ++g) {
    const int64_t ib = ni * g / groups, ie = ni * (g + 1) / groups;
    for (int64_t i = ib; i < ie;) {
      const int32_t o = it[4 * i];
      int64_t j = i;
      while (j < ie && it[4 * j] == o) ++j;
      const int32_t next = j < ie ? it[4 * j] + 1 : 0;  // next segment's offset + 1
      for (int64_t r = i; r < j; r += 4)
        for (int w = 0; w < 4; ++w) {
          const int64_t q = r + w;
          P.rounds.push_back(o);
          P.rounds.push_back(q < j ? it[4 * q + 1] : 0);
          P.rounds.push_back(q < j ? it[4 * q + 2] : 0);
          P.rounds.push_back(r == i ? (1 | (next << 1)) : 0);
        }
      i = j;
    }
    P.wg_round_ptr[g + 1] = (int32_t)(P.rounds.size() / 16);
  }
}

int64_t max_rounds(const Plan& p) {
  // ceil(items / 4) rounds, plus at most one partial round per segment;
  // segments are runs of one offset cut at most once per workgroup
  return p.n_items() / 4 + p.n_off() + kMaxTranslateGroups + 1;
}

Layout workspace_layout(const Plan& p, int32_t max_nrhs) {
  Layout L{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t here = at;
    at = align256(at + bytes);
    return here;
  };
  L.table = take(p.table_bytes());
  L.chunks = take(p.chunks.size() * sizeof(int32_t));
  L.items = take(p.items.size() * sizeof(int32_t));
  L.wg_ptr = take((size_t)(kMaxTranslateGroups + 1) * sizeof(int32_t));
  L.rounds = take((size_t)max_rounds(p) * 16 * sizeof(int32_t));
  L.wg_round_ptr = take((size_t)(kMaxTranslateGroups + 1) * sizeof(int32_t));
  L.pair_src = take(p.pair_src.size() * sizeof(int32_t));
  L.pair_dst = take(p.pair_dst.size() * sizeof(int32_t));
  L.test_ptr = take(p.test_ptr.size() * sizeof(int32_t));
  L.nb_ptr = take((size_t)(p.n_box + 1) * sizeof(int64_t));
  L.P = take((size_t)max_nrhs * p.n_box * p.vstride() * sizeof(float));
  // one spare row at the end receives the stores of idle matrix-core lanes
  L.part = take(((size_t)max_nrhs * p.n_pairs() + 1) * p.pstride() * sizeof(float));
  L.off_scale = take((size_t)std::max<int32_t>(p.n_off(), 1) * sizeof(float));
  L.box_scale = take((size_t)max_nrhs * p.n_box * sizeof(float));
  L.offsets = take(p.offsets.size() * sizeof(int32_t));
  L.total = at;
  return L;
}

ScratchLayout scratch_layout(const Plan& p, int32_t nrhs) {
  ScratchLayout L{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t here = at;
    at = align256(at + bytes);
    return here;
  };
  L.P = take((size_t)nrhs * p.n_box * p.vstride() * sizeof(float));
  L.part = take(((size_t)nrhs * p.n_pairs() + 1) * p.pstride() * sizeof(float));
  L.box_scale = take((size_t)nrhs * p.n_box * sizeof(float));
  L.total = at;
  return L;
}

std::string build_plan(const int32_t* box_ijk, int64_t n_box, double a,
                       double k, double eta, int n_d, int far_mode,
                       int precision, int operators, const int64_t* scat_ptr,
                       int64_t n_scat, Plan& P) {
  if (!box_ijk) return "box_ijk is NULL";
  if (n_box < 1) return "n_boxes must be >= 1";
  if (n_box > std::numeric_limits<int32_t>::max() / 2) return "n_boxes too large";
  if (!(a > 0.0) || !std::isfinite(a)) return "box side a must be > 0";
  if (!(k > 0.0) || !std::isfinite(k)) return "wavenumber k must be > 0";
  if (!(eta >= 0.0) || !std::isfinite(eta)) return "eta must be >= 0 (0 = free space)";
  if (n_d < 1 || n_d > 4) return "n_d must be in 1..4";
  if (far_mode != 0 && far_mode != 1) return "unknown far_mode";
  if (precision < 0 || precision > 3) return "unknown precision";
  if (operators != 0 && operators != 1) return "unknown operator source";
  if (operators == 1 && (precision == 0 || n_d > 3))
    return "generated operators need a 16-bit form (precision 1..3) and n_d 1..3";

  P.n_box = n_box;
  P.boxes.assign(box_ijk, box_ijk + 3 * n_box);
  for (int64_t i = 0; i < 3 * n_box; ++i)
    if (P.boxes[i] < 0) return "box coordinates must be >= 0";
  P.a = a;
  P.k = k;
  P.eta = eta == 0.0 ? kEta0 : eta;
  P.n_d = n_d;
  P.nu = 3 * n_d * n_d * n_d;
  P.kh = half_len(P.nu);
  P.khb = half_len_bf16(P.nu);
  P.far_mode = far_mode;
  P.precision = precision;
  P.gen_ops = operators == 1;

  if (scat_ptr) {
    if (n_scat < 1) return "n_scatterers must be >= 1";
    if (scat_ptr[0] != 0) return "scatterer_ptr[0] must be 0";
    for (int64_t s = 0; s < n_scat; ++s)
      if (scat_ptr[s + 1] <= scat_ptr[s]) return "every scatterer needs at least one box";
    if (scat_ptr[n_scat] != n_box) return "scatterer_ptr[n_scatterers] must equal n_boxes";
    P.scat_ptr.assign(scat_ptr, scat_ptr + n_scat + 1);
  } else {
    P.scat_ptr = {0, n_box};
  }
  const int32_t* b = P.boxes.data();

  // Far set: (test j, source i, offset w = c_j - c_i), test-major, built
  // within each scatterer (global box indices).
  std::vector<int32_t> pj, pi;
  std::vector<std::array<int32_t, 3>> pw;
  const int64_t kMaxPairs = std::numeric_limits<int32_t>::max();
  BoxIndex index;
  for (int64_t sc = 0; sc + 1 < (int64_t)P.scat_ptr.size(); ++sc) {
    const int64_t lo = P.scat_ptr[sc], hi = P.scat_ptr[sc + 1];
    if (!index.build(b + 3 * lo, hi - lo)) return "duplicate box coordinates";
    if (far_mode == 0) {
      for (int64_t j = lo; j < hi; ++j) {
        const int64_t cx = b[3 * j], cy = b[3 * j + 1], cz = b[3 * j + 2];
        for (int wx = -3; wx <= 3; ++wx)
          for (int wy = -3; wy <= 3; ++wy)
            for (int wz = -3; wz <= 3; ++wz) {
              if (cheb(wx, wy, wz) < 2) continue;
              const int64_t sx = cx - wx, sy = cy - wy, sz = cz - wz;
              const int32_t il = index.find(sx, sy, sz);
              if (il < 0) continue;
              if (cheb(floordiv2(cx) - floordiv2(sx), floordiv2(cy) - floordiv2(sy),
                       floordiv2(cz) - floordiv2(sz)) > 1)
                continue;
              if ((int64_t)pj.size() >= kMaxPairs) return "far set exceeds 2^31-1 pairs";
              pj.push_back((int32_t)j);
              pi.push_back((int32_t)(lo + il));
              pw.push_back({wx, wy, wz});
            }
      }
    } else {
      for (int64_t j = lo; j < hi; ++j)
        for (int64_t i = lo; i < hi; ++i) {
          const int64_t wx = (int64_t)b[3 * j] - b[3 * i];
          const int64_t wy = (int64_t)b[3 * j + 1] - b[3 * i + 1];
          const int64_t wz = (int64_t)b[3 * j + 2] - b[3 * i + 2];
          if (cheb(wx, wy, wz) < 2) continue;
          if ((int64_t)pj.size() >= kMaxPairs) return "far set exceeds 2^31-1 pairs";
          pj.push_back((int32_t)j);
          pi.push_back((int32_t)i);
          pw.push_back({(int32_t)wx, (int32_t)wy, (int32_t)wz});
        }
    }
  }
  if ((int64_t)pj.size() > kMaxPairs) return "far set exceeds 2^31-1 pairs";

  // Distinct offsets, lexicographic: collect them through a hash of the
  // pairs' offsets (far fewer than pairs), sort only those, then map.
  const int64_t np = (int64_t)pj.size();
  std::vector<int32_t> oid(np);
  std::vector<std::array<int32_t, 3>> uniq;
  {
    struct Hash {
      size_t operator()(const std::array<int32_t, 3>& w) const {
        uint64_t h = (uint32_t)w[0];
        h = h * 0x9E3779B97F4A7C15ull ^ (uint32_t)w[1];
        h = h * 0x9E3779B97F4A7C15ull ^ (uint32_t)w[2];
        return (size_t)(h ^ (h >> 29));
      }
    };
    std::unordered_map<std::array<int32_t, 3>, int32_t, Hash> seen;
    for (int64_t p = 0; p < np; ++p) {
      auto it = seen.find(pw[p]);
      if (it == seen.end()) {
        it = seen.emplace(pw[p], (int32_t)uniq.size()).first;
        uniq.push_back(pw[p]);
      }
      oid[p] = it->second;
    }
    std::vector<int32_t> order(uniq.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int32_t x, int32_t y) { return uniq[x] < uniq[y]; });
    std::vector<int32_t> rank(uniq.size());
    std::vector<std::array<int32_t, 3>> sorted(uniq.size());
    for (size_t r = 0; r < order.size(); ++r) {
      rank[order[r]] = (int32_t)r;
      sorted[r] = uniq[order[r]];
    }
    uniq.swap(sorted);
    for (int64_t p = 0; p < np; ++p) oid[p] = rank[oid[p]];
  }
  const int64_t n_off = (int64_t)uniq.size();
  // bytes of one offset's image in the table layout of the plan's form
  const size_t img_bytes = P.staged_split() ? P.staged_split_halves() * sizeof(uint16_t)
                           : P.split()        ? (size_t)4 * P.nu * P.khb * sizeof(uint16_t)
                           : P.staged()       ? P.staged_op_floats() * sizeof(float)
                                              : (size_t)2 * P.nu * P.kh * sizeof(float);
  if (!P.gen_ops && (double)n_off * (double)img_bytes > kMaxTableBytes)
    return "operator table would exceed 16 GiB";
  P.offsets.resize(3 * n_off);
  for (int64_t o = 0; o < n_off; ++o)
    for (int d = 0; d < 3; ++d) P.offsets[3 * o + d] = uniq[o][d];

  // Stable counting sort of the pairs by offset.
  P.off_ptr.assign(n_off + 1, 0);
  for (int64_t p = 0; p < np; ++p) P.off_ptr[oid[p] + 1]++;
  for (int64_t o = 0; o < n_off; ++o) P.off_ptr[o + 1] += P.off_ptr[o];
  std::vector<int64_t> fill(P.off_ptr.begin(), P.off_ptr.end() - 1);
  P.pair_test.resize(np);
  P.pair_src.resize(np);
  P.pair_off.resize(np);
  for (int64_t p = 0; p < np; ++p) {
    const int64_t at = fill[oid[p]]++;
    P.pair_test[at] = pj[p];
    P.pair_src[at] = pi[p];
    P.pair_off[at] = oid[p];
  }

  // Test box -> positions of its pairs in the grouped order.
  P.test_ptr.assign(n_box + 1, 0);
  for (int64_t p = 0; p < np; ++p) P.test_ptr[P.pair_test[p] + 1]++;
  for (int64_t j = 0; j < n_box; ++j) P.test_ptr[j + 1] += P.test_ptr[j];
  std::vector<int32_t> tfill(P.test_ptr.begin(), P.test_ptr.end() - 1);
  P.test_pos.resize(np);
  for (int64_t p = 0; p < np; ++p) P.test_pos[tfill[P.pair_test[p]]++] = (int32_t)p;
  // Partial products are written at their test-major position, so the
  // pairs of one test box occupy consecutive rows.
  P.pair_dst.resize(np);
  for (int64_t q = 0; q < np; ++q) P.pair_dst[P.test_pos[q]] = (int32_t)q;

  // Work units: up to kChunk consecutive pairs of one offset.
  P.chunks.clear();
  for (int64_t o = 0; o < n_off; ++o)
    for (int64_t s = P.off_ptr[o]; s < P.off_ptr[o + 1]; s += kChunk) {
      P.chunks.push_back((int32_t)o);
      P.chunks.push_back((int32_t)s);
      P.chunks.push_back((int32_t)std::min<int64_t>(kChunk, P.off_ptr[o + 1] - s));
      P.chunks.push_back(0);
    }
  P.items.clear();
  for (int64_t o = 0; o < n_off; ++o)
    for (int64_t s = P.off_ptr[o]; s < P.off_ptr[o + 1]; s += 32) {
      P.items.push_back((int32_t)o);
      P.items.push_back((int32_t)s);
      P.items.push_back((int32_t)std::min<int64_t>(32, P.off_ptr[o + 1] - s));
      P.items.push_back(0);
    }

  partition_groups(P, kTranslateGroups);
  build_rounds(P, kRoundGroups);

  // Orbits under the 48 signed permutations: key = sorted |w|.
  std::vector<std::array<int32_t, 3>> keys(n_off);
  for (int64_t o = 0; o < n_off; ++o) {
    std::array<int32_t, 3> kk = {std::abs(uniq[o][0]), std::abs(uniq[o][1]),
                                 std::abs(uniq[o][2])};
    std::sort(kk.begin(), kk.end());
    keys[o] = kk;
  }
  std::sort(keys.begin(), keys.end());
  P.n_orbits = (int32_t)(std::unique(keys.begin(), keys.end()) - keys.begin());

  P.off_scale.assign(n_off, 1.0f);
  if (P.gen_ops) return std::string();  // evaluated by the translation kernel

  // Operator table image, one offset at a time (cached across plans).
  if (P.split())
    P.table_bf16.assign((size_t)n_off * img_bytes / sizeof(uint16_t), 0);
  else
    P.table.assign((size_t)n_off * img_bytes / sizeof(float), 0.0f);
  char* table = P.split() ? (char*)P.table_bf16.data() : (char*)P.table.data();
  // Offsets are independent: large tables (FULL far sets have one operator
  // per distinct offset, ~10^5 on a few-thousand-box scatterer) are built
  // on several host threads, each over a contiguous range of offsets.
  auto build_range = [&](int64_t lo, int64_t hi) {
    std::vector<std::complex<double>> G;
    for (int64_t o = lo; o < hi; ++o) {
      char* dst = table + (size_t)o * img_bytes;
      if (!image_cache_get(P, &P.offsets[3 * o], dst, img_bytes, &P.off_scale[o])) {
        offset_image(P, &P.offsets[3 * o], G, dst, &P.off_scale[o]);
        image_cache_put(P, &P.offsets[3 * o], dst, img_bytes, P.off_scale[o]);
      }
    }
  };
  const int64_t kPerThread = 1024;
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int64_t nthr = std::min<int64_t>(std::min(hw, 16), (n_off + kPerThread - 1) / kPerThread);
  if (nthr <= 1) {
    build_range(0, n_off);
  } else {
    std::vector<std::thread> pool;
    for (int64_t t = 0; t < nthr; ++t)
      pool.emplace_back(build_range, n_off * t / nthr, n_off * (t + 1) / nthr);
    for (auto& th : pool) th.join();
  }
  return std::string();
}

}  // namespace ubf

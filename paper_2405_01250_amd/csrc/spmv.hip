// spmv.hip -- DiaQ sparse matrix-vector product (Alg. 2) and the fused
// expectation / generator reductions, for gfx950.
//
// Row ownership replaces Alg. 2's loop over diagonals: each lane owns output
// rows and sums, in ascending diagonal index, D_k(i) * x[i + d_k] over the
// diagonals whose range covers row i, then stores y[i] once.  There is one
// writer per y element, so the race of Alg. 2's parallel loop over
// diagonals (all writing y) cannot occur, no atomics are needed and y is
// never read or pre-zeroed.
//
// Memory plan (the product is HBM-bound, ~0.3 flop/byte in fp64):
//  * a wave reads 64 consecutive rows, so every diagonal stream and every
//    shifted x stream is a unit-stride, 16-byte-per-lane coalesced access;
//  * on matrices expanded from a gate or a Pauli sum, a value that is
//    exactly zero skips its x load: such zeros are structural (half of each
//    off-principal diagonal of an expanded one-qubit gate lies outside the
//    gate's coupling), and skipping them keeps x at one HBM read per
//    element.  Every other matrix multiplies each stored element with its
//    x entry, zeros included, so a non-finite x reaches y as Alg. 2 has it
//    (0 * Inf = NaN);
//  * offsets larger than a tile are handled by grouping tiles: one
//    workgroup owns the tiles {base + sum s_b 2^b} for the gate's high
//    coupling bits b, so x[i] and x[i +- 2^b] are fetched from HBM once and
//    re-read from L1/L2 of the same CU (workgroups are spread round-robin
//    over the 8 XCDs, so sharing across workgroups would not hit one L2).
#include <mutex>

#include "internal.hpp"

// Per-workgroup partial sums of the allocation-free expectation
// (diaq_expect_noalloc): kStaticPartials entries, 16 MiB, enough for the
// product of a 2^28-row matrix at one row per lane.  Each device holds its
// own copy until the process ends.  In host code this name is only a
// host-side stand-in: kernels receive the device address that
// init_static_scratch takes with hipGetSymbolAddress.
static __device__ __align__(256) double2 scratch[diaq::kStaticPartials];

namespace diaq {

namespace {

constexpr int kBlock = 256;

template <typename R>
struct Vec;
template <>
struct Vec<double> {
  using V = double2;
};
template <>
struct Vec<float> {
  using V = float2;
};
// Two consecutive complex64 amplitudes as one 16-byte unit (re0, im0, re1,
// im1): complex64 products whose offsets and diagonal starts are all even
// run on N / 2 units with halved offsets, so every state and diagonal
// access is 16 bytes per lane, as in complex128 (8-byte accesses stream
// more slowly; n = 28, mean over target qubits: U3 5.89 -> 6.13 TB/s, CX
// 5.90 -> 6.16, diagonal gates 5.97 -> 6.36).  Each amplitude's sum is
// formed as in the unpacked product, so the two agree exactly.
struct Pk {};
template <>
struct Vec<Pk> {
  using V = float4;
};

struct RowMap {
  int64_t N;
  int32_t tile_log2;  // log2(rows per tile)
  int32_t ng;         // number of group bits (0..3)
  int32_t gbit[3];    // ascending qubit indices, each >= tile_log2
  int32_t run_log2;   // XCD runs of 2^run_log2 tiles (0: launch order)
  int32_t pair_bit;   // > 0: each XCD alternates between tiles differing in this tile bit
  int32_t order;      // otherwise: 1 XCD-contiguous eighths, 2 halves interleaved
};

// Tile of workgroup b.  The device hands consecutive workgroups to its 8
// XCDs in turn, and each XCD has its own L2, so a tile whose partner rows
// sit 1, 2 or 4 tiles away would fetch them through another XCD's cache.
// With run_log2 = r each XCD takes runs of 2^r consecutive tiles (chunks of
// 8 runs; the last partial chunk keeps launch order), and a tile meets its
// partner less than 2^r tiles away in the same L2.
__device__ __forceinline__ int64_t tile_of(int64_t b, const RowMap& m) {
  if (m.pair_bit > 0) {
    // consecutive workgroups of one XCD take a tile and its partner 2^p
    // tiles away; the last partial group of 16 keeps launch order
    const int64_t nb = int64_t(gridDim.x);
    if (b >= (nb / 16) * 16) return b;
    const int64_t x = b & 7, u = b >> 3;
    const int64_t c = ((u >> 1) << 3) | x;
    const int p = m.pair_bit;
    return ((c >> p) << (p + 1)) | ((u & 1) << p) | (c & ((int64_t(1) << p) - 1));
  }
  if (m.run_log2 == 0) {
    const int64_t nb = int64_t(gridDim.x);
    if (m.order == 1 && (nb & 7) == 0) return (b & 7) * (nb >> 3) + (b >> 3);
    if (m.order == 2 && (nb & 1) == 0) return (b >> 1) + (b & 1) * (nb >> 1);
    return b;
  }
  const int64_t w = int64_t(1) << m.run_log2, chunk = 8 * w;
  if (b >= (int64_t(gridDim.x) / chunk) * chunk) return b;
  const int64_t in = b % chunk;
  return (b - in) + (in % 8) * w + in / 8;
}

// Insert a zero bit at each group position (ascending) into v.
__device__ __forceinline__ int64_t insert_zero_bits(int64_t v, const RowMap& m) {
  for (int b = 0; b < m.ng; b++) {
    const int p = m.gbit[b];
    const int64_t lo = v & ((int64_t(1) << p) - 1);
    v = lo | ((v >> p) << (p + 1));
  }
  return v;
}

__device__ __forceinline__ int64_t group_offset(int s, const RowMap& m) {
  int64_t o = 0;
  for (int b = 0; b < m.ng; b++)
    if ((s >> b) & 1) o |= int64_t(1) << m.gbit[b];
  return o;
}

struct DiagSrc {
  const int64_t* dmeta;  // device table or nullptr
  int32_t nd;
  int32_t transpose;
  int32_t conjugate;
  int32_t skip_zero;     // zero values are structural: skip their x loads
};

// (applied offset e, value base vb): row i uses vals[vb + i] * x[i + e].
// DM selects the device table (matrices with many diagonals) over the
// kernel-argument copy; both are uniform, scalar-loaded reads.
template <bool DM>
__device__ __forceinline__ void diag_at(const DiagArgs& da, const DiagSrc& src, int k,
                                        int64_t& e, int64_t& vb) {
  const int kk = src.transpose ? (src.nd - 1 - k) : k;
  int64_t d, st;
  if constexpr (DM) {
    d = src.dmeta[kk];
    st = src.dmeta[src.nd + kk];
  } else {
    d = da.off[kk];
    st = da.start[kk];
  }
  if (src.transpose) {
    // (A^T) diagonal -d at row i is A's diagonal d at row i - d, whose
    // compact index is (i - d) + min(0, d) = i - max(0, d).
    e = -d;
    vb = st - (d > 0 ? d : 0);
  } else {
    e = d;
    vb = st + (d < 0 ? d : 0);
  }
}

template <typename V>
__device__ __forceinline__ bool nonzero(const V& v) {
  if constexpr (std::is_same<V, float4>::value) return v.x != 0 || v.y != 0 || v.z != 0 || v.w != 0;
  else return v.x != 0 || v.y != 0;
}

// A packed unit's x entries behind a structural zero value stay zero (as
// the skipped load leaves them in the unpacked product), so a non-finite x
// there does not reach y.
template <typename V>
__device__ __forceinline__ void drop_behind_zeros(V& xv, const V& v) {
  if constexpr (std::is_same<V, float4>::value) {
    if (v.x == 0 && v.y == 0) xv.x = xv.y = 0;
    if (v.z == 0 && v.w == 0) xv.z = xv.w = 0;
  }
}

template <typename R>
__device__ __forceinline__ void cfma(typename Vec<R>::V& acc, const typename Vec<R>::V& a,
                                     const typename Vec<R>::V& b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  if constexpr (std::is_same<R, Pk>::value) {
    acc.z = fma(a.z, b.z, acc.z);
    acc.z = fma(-a.w, b.w, acc.z);
    acc.w = fma(a.z, b.w, acc.w);
    acc.w = fma(a.w, b.z, acc.w);
  }
}

template <typename V>
__device__ __forceinline__ V vzero() {
  V v;
  v.x = 0;
  v.y = 0;
  if constexpr (std::is_same<V, float4>::value) {
    v.z = 0;
    v.w = 0;
  }
  return v;
}

template <typename V>
__device__ __forceinline__ void vconj(V& v) {
  v.y = -v.y;
  if constexpr (std::is_same<V, float4>::value) v.w = -v.w;
}

template <typename V>
struct NativeT {
  using T = typename HIP_vector_base<decltype(V{}.x), 2>::Native_vec_;
};
template <>
struct NativeT<float4> {
  typedef float T __attribute__((ext_vector_type(4)));
};
template <typename V>
using NativeOf = typename NativeT<V>::T;

template <bool NT, typename V>
__device__ __forceinline__ V ld(const V* p) {
  if constexpr (NT) {
    const auto t = __builtin_nontemporal_load(reinterpret_cast<const NativeOf<V>*>(p));
    if constexpr (std::is_same<V, float4>::value) return V{t[0], t[1], t[2], t[3]};
    else return V{t[0], t[1]};
  } else {
    return *p;
  }
}

template <bool NT, typename V>
__device__ __forceinline__ void st(V* p, const V& v) {
  if constexpr (NT) {
    NativeOf<V> t;
    t[0] = v.x;
    t[1] = v.y;
    if constexpr (std::is_same<V, float4>::value) {
      t[2] = v.z;
      t[3] = v.w;
    }
    __builtin_nontemporal_store(t, reinterpret_cast<NativeOf<V>*>(p));
  } else {
    *p = v;
  }
}

// Computes acc[s*RPT + j] = (op(A) x)[row(s, j)] for the G*RPT rows a lane
// owns; rows outside [0, N) (only when N < tile) are left at zero.
// Diagonals are taken KC at a time: all their values are loaded, then all
// the x loads they need are issued, then the multiplies run, so the x
// elements that paired rows share are requested back to back.  NT marks
// the single-use value stream non-temporal.
template <typename R, int RPT, int G, bool CHECK, int KC, bool NT, bool DM>
__device__ __forceinline__ void dia_rows(const DiagArgs& da, const DiagSrc& src, const RowMap& m,
                                         const typename Vec<R>::V* __restrict__ vals,
                                         const typename Vec<R>::V* __restrict__ x, int64_t base,
                                         typename Vec<R>::V (&acc)[G * RPT],
                                         int64_t (&row)[G * RPT]) {
  using V = typename Vec<R>::V;
  constexpr int ROWS = G * RPT;
  const int64_t N = m.N;
#pragma unroll
  for (int s = 0; s < G; s++)
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      row[s * RPT + j] = base + group_offset(s, m) + j * kBlock + threadIdx.x;
      acc[s * RPT + j] = vzero<V>();
    }
  for (int k0 = 0; k0 < src.nd; k0 += KC) {
    // the chunk's diagonal descriptors first, so no value load waits on them
    int64_t ek[KC], vbk[KC], lok[KC], hik[KC];
#pragma unroll
    for (int c = 0; c < KC; c++) {
      int64_t e = 0, vb = 0;
      if ((k0 + c) < src.nd) diag_at<DM>(da, src, k0 + c, e, vb);
      ek[c] = e;
      vbk[c] = vb;
      lok[c] = (k0 + c) < src.nd ? (e < 0 ? -e : 0) : N;
      hik[c] = e > 0 ? N - e : N;
    }
    V v[KC][ROWS];
    bool in[KC][ROWS];
#pragma unroll
    for (int c = 0; c < KC; c++) {
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        const int64_t i = row[r];
        in[c][r] = (i >= lok[c]) && (i < hik[c]) && (!CHECK || i < N);
        v[c][r] = in[c][r] ? ld<NT>(vals + vbk[c] + i) : vzero<V>();
      }
    }
    if (src.conjugate) {
#pragma unroll
      for (int c = 0; c < KC; c++)
#pragma unroll
        for (int r = 0; r < ROWS; r++) vconj(v[c][r]);
    }
    // issue every x load of the chunk before the first multiply
    V xv[KC][ROWS];
#pragma unroll
    for (int c = 0; c < KC; c++)
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        xv[c][r] = vzero<V>();
        if (in[c][r] && (!src.skip_zero || nonzero(v[c][r]))) xv[c][r] = x[row[r] + ek[c]];
        if (src.skip_zero) drop_behind_zeros(xv[c][r], v[c][r]);
      }
    // ascending diagonal order within every row
#pragma unroll
    for (int c = 0; c < KC; c++)
#pragma unroll
      for (int r = 0; r < ROWS; r++) cfma<R>(acc[r], v[c][r], xv[c][r]);
  }
}

template <typename R, int RPT, int G, bool CHECK, int KC, bool NT, bool DM>
__global__ __launch_bounds__(kBlock) void spmv_kernel(DiagArgs da, DiagSrc src, RowMap m,
                                                      const typename Vec<R>::V* __restrict__ vals,
                                                      const typename Vec<R>::V* __restrict__ x,
                                                      typename Vec<R>::V* __restrict__ y) {
  using V = typename Vec<R>::V;
  const int64_t base = insert_zero_bits(tile_of(int64_t(blockIdx.x), m) << m.tile_log2, m);
  V acc[G * RPT];
  int64_t row[G * RPT];
  dia_rows<R, RPT, G, CHECK, KC, NT, DM>(da, src, m, vals, x, base, acc, row);
#pragma unroll
  for (int r = 0; r < G * RPT; r++)
    if (!CHECK || row[r] < m.N) st<NT>(y + row[r], acc[r]);
}

// In-place variant for matrices whose only diagonal is the principal one.
template <typename R, bool NT>
__global__ __launch_bounds__(kBlock) void diag_inplace_kernel(int64_t N, int32_t conjugate,
                                                              const typename Vec<R>::V* __restrict__ vals,
                                                              typename Vec<R>::V* xy) {
  using V = typename Vec<R>::V;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += stride) {
    V v = ld<NT>(vals + i);
    if (conjugate) vconj(v);
    const V a = ld<NT>(xy + i);
    V r = vzero<V>();
    cfma<R>(r, v, a);
    st<NT>(xy + i, r);
  }
}

// ---------------------------------------------------------------------------
// Reductions: per-workgroup partial sums in fixed order, then one pass.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void block_reduce_store(double re, double im, double2* partial) {
  // wave64 butterfly
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  __shared__ double2 wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wsum[wave] = double2{re, im};
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 t = wsum[0];
    for (int w = 1; w < kBlock / 64; w++) {
      t.x += wsum[w].x;
      t.y += wsum[w].y;
    }
    partial[blockIdx.x] = t;
  }
}

template <typename R, int RPT, int G, bool CHECK, int KC, bool NT, bool DM>
__global__ __launch_bounds__(kBlock) void expect_kernel(DiagArgs da, DiagSrc src, RowMap m,
                                                        const typename Vec<R>::V* __restrict__ vals,
                                                        const typename Vec<R>::V* __restrict__ psi,
                                                        const typename Vec<R>::V* __restrict__ phi,
                                                        double2* __restrict__ partial) {
  using V = typename Vec<R>::V;
  const int64_t base = insert_zero_bits(tile_of(int64_t(blockIdx.x), m) << m.tile_log2, m);
  V acc[G * RPT];
  int64_t row[G * RPT];
  dia_rows<R, RPT, G, CHECK, KC, NT, DM>(da, src, m, vals, phi, base, acc, row);
  double re = 0, im = 0;
#pragma unroll
  for (int r = 0; r < G * RPT; r++) {
    if (CHECK && row[r] >= m.N) continue;
    const V p = psi[row[r]];
    // conj(p) * acc
    re += double(p.x) * double(acc[r].x) + double(p.y) * double(acc[r].y);
    im += double(p.x) * double(acc[r].y) - double(p.y) * double(acc[r].x);
  }
  block_reduce_store(re, im, partial);
}

// One workgroup sums partial[0..count) in a fixed order.
__global__ __launch_bounds__(1024) void final_reduce_kernel(const double2* __restrict__ partial,
                                                            int64_t count, double2* __restrict__ out) {
  double re = 0, im = 0;
  for (int64_t i = threadIdx.x; i < count; i += 1024) {
    re += partial[i].x;
    im += partial[i].y;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  __shared__ double2 wsum[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wsum[wave] = double2{re, im};
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 t = wsum[0];
    for (int w = 1; w < 16; w++) {
      t.x += wsum[w].x;
      t.y += wsum[w].y;
    }
    *out = t;
  }
}

// <lam | G | psi> where G acts on k target qubits (local matrix gm) and is
// zero wherever a control bit is 0.  Each lane owns one coset of 2^k
// amplitudes (the target bits enumerate it), so lam and psi are read once.
struct GenArgs {
  int64_t ncos;         // number of cosets = N / 2^k
  int32_t k;
  int32_t tq[3];        // target qubits, ascending order of local bit
  int32_t sorted_t[3];  // target qubits sorted ascending (for insertion)
  uint64_t cmask;
  double g[8][8][2];
};

template <typename R>
__global__ __launch_bounds__(kBlock) void generator_dot_kernel(GenArgs a,
                                                               const typename Vec<R>::V* __restrict__ lam,
                                                               const typename Vec<R>::V* __restrict__ psi,
                                                               double2* __restrict__ partial) {
  using V = typename Vec<R>::V;
  double re = 0, im = 0;
  const int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (c < a.ncos) {
    int64_t b = c;
    for (int j = 0; j < a.k; j++) {
      const int p = a.sorted_t[j];
      b = (b & ((int64_t(1) << p) - 1)) | ((b >> p) << (p + 1));
    }
    if ((uint64_t(b) & a.cmask) == a.cmask) {
      const int d = 1 << a.k;
      int64_t idx[8];
      double pr[8], pi[8];
      for (int r = 0; r < d; r++) {
        int64_t o = 0;
        for (int j = 0; j < a.k; j++)
          if ((r >> j) & 1) o |= int64_t(1) << a.tq[j];
        idx[r] = b + o;
        const V p = psi[idx[r]];
        pr[r] = p.x;
        pi[r] = p.y;
      }
      for (int r = 0; r < d; r++) {
        double gr = 0, gi = 0;
        for (int cc = 0; cc < d; cc++) {
          const double mr = a.g[r][cc][0], mi = a.g[r][cc][1];
          gr += mr * pr[cc] - mi * pi[cc];
          gi += mr * pi[cc] + mi * pr[cc];
        }
        const V l = lam[idx[r]];
        re += double(l.x) * gr + double(l.y) * gi;
        im += double(l.x) * gi - double(l.y) * gr;
      }
    }
  }
  block_reduce_store(re, im, partial);
}

// ---------------------------------------------------------------------------
// Host planning
// ---------------------------------------------------------------------------

struct Plan {
  RowMap map;
  int rpt;
  int g;
  int kc;
  bool nt;
  bool check;
  int64_t blocks;
};

// Row tiling and kernel variant.  Defaults (measured on MI355X at n = 28,
// one-qubit gates on every qubit): 1 row per lane per tile, tiles paired
// over up to 3 coupling qubits >= 21 (partners closer than that meet in the
// 256 MB last-level cache anyway), one diagonal's loads at a time, and
// non-temporal value / y streams so they do not evict x.
constexpr int kDefaultRows = 1;
constexpr int kDefaultGroupMinQubit = 21;

// Partner distance from which far partners are alternated on each XCD:
// in launch order an XCD reaches a tile's partner D / 8 workgroups later,
// after about 5 D / 8 tiles of other traffic, which its 4 MB L2 holds up to
// partners about 16 MiB apart (measured: alternating is slower below that,
// up to 1.2x faster beyond).
constexpr int64_t kPairOrderMinBytes = int64_t(16) << 20;

Plan plan_rows(const SpmvOp& op, const diaq_tuning_t& t, int rpt_override) {
  Plan p{};
  const int n = op.n;
  p.map.N = int64_t(1) << n;
  int rpt = rpt_override > 0 ? rpt_override : (t.spmv_rows > 0 ? t.spmv_rows : kDefaultRows);
  if (rpt != 1 && rpt != 2 && rpt != 4) rpt = kDefaultRows;
  // with packing on, the rows knob counts 16-byte units (two complex64
  // amplitudes): a complex64 product that cannot be packed takes twice as
  // many rows per lane, the same bytes
  if (op.dtype == DIAQ_C64 && t.spmv_pack >= 0 && rpt_override <= 0) rpt = std::min(4, 2 * rpt);
  int max_bits = t.spmv_group_bits < 0 ? 0 : (t.spmv_group_bits == 0 ? 3 : std::min(3, t.spmv_group_bits));
  if (op.nd > kMaxArgDiags) {
    // descriptor-table kernels come in one shape: 2 rows per lane, no grouping
    rpt = 2;
    max_bits = 0;
  }
  p.kc = (t.spmv_chunk == 3) ? 3 : 1;
  p.nt = t.spmv_nontemporal >= 0;
  int tile_log2 = 8 + (rpt == 4 ? 2 : rpt == 2 ? 1 : 0);
  if (n < tile_log2) {
    // tiny matrix: one row per lane, bounds-checked
    p.rpt = 1;
    p.g = 1;
    p.check = true;
    p.map.tile_log2 = 8;
    p.map.ng = 0;
    p.blocks = (p.map.N + kBlock - 1) / kBlock;
    return p;
  }
  // group the highest coupling bits at or above the tile size
  int bits[64], nb = 0;
  const int qmin =
      std::max(tile_log2, t.spmv_group_min_qubit > 0 ? t.spmv_group_min_qubit : kDefaultGroupMinQubit);
  if (t.spmv_group_qubits) {
    // per-qubit choice (autotuned): pair across the chosen coupling qubits
    for (int q = n - 1; q >= tile_log2 && nb < max_bits; q--)
      if (((op.qubit_mask & t.spmv_group_qubits) >> q) & 1) bits[nb++] = q;
  } else {
    for (int q = n - 1; q >= qmin && nb < max_bits; q--)
      if ((op.qubit_mask >> q) & 1) bits[nb++] = q;
  }
  // at most 4 rows per lane: larger groups take fewer rows per tile
  while ((rpt << nb) > 4 && rpt > 1) {
    rpt >>= 1;
    tile_log2--;
  }
  if ((rpt << nb) > 4) p.kc = 1;  // G = 8: keep the register budget
  p.rpt = rpt;
  p.map.tile_log2 = tile_log2;
  p.map.ng = nb;
  for (int b = 0; b < nb; b++) p.map.gbit[b] = bits[nb - 1 - b];  // ascending
  p.g = 1 << nb;
  p.check = false;
  p.blocks = p.map.N >> (tile_log2 + nb);
  // XCD runs, for matrices whose every off-tile diagonal couples tiles 1, 2
  // or 4 apart (a gate on qubit tile_log2 .. tile_log2 + 2): runs twice
  // the largest such distance; any other distance keeps launch order,
  // which already keeps distances that are multiples of 8 on one XCD
  if (nb == 0 && op.nd <= kMaxArgDiags && t.spmv_xcd_runs >= 0) {
    int64_t dmax = 0;
    bool plain = true;
    const int64_t tile = int64_t(1) << tile_log2;
    for (int k = 0; k < op.nd; k++) {
      const int64_t d = op.host_off[k] < 0 ? -op.host_off[k] : op.host_off[k];
      if (d < tile) continue;
      const int64_t dt = d / tile;
      if (d % tile != 0 || dt >= 8 || (dt & (dt - 1)) != 0) plain = false;
      dmax = std::max(dmax, dt);
    }
    if (plain && dmax > 0) {
      const int r = dmax == 1 ? 1 : dmax == 2 ? 2 : 3;
      if (p.blocks >= (int64_t(8) << r)) p.map.run_log2 = r;
    }
  }
  // far partners (one coupling qubit whose tiles are >= 2^3 apart, not
  // paired inside a workgroup): alternate partner tiles on each XCD
  if (nb == 0 && op.nd <= kMaxArgDiags && t.spmv_xcd_runs >= 0 && p.map.run_log2 == 0) {
    int pb = -1, cnt = 0;
    for (int q = tile_log2 + 3; q < n; q++)
      if ((op.qubit_mask >> q) & 1) {
        pb = q - tile_log2;
        cnt++;
      }
    int low = 0;
    for (int q = 0; q < tile_log2 + 3 && q < n; q++) low += ((op.qubit_mask >> q) & 1) && q >= tile_log2 ? 1 : 0;
    const int64_t tile_bytes = (int64_t(1) << tile_log2) * int64_t(elem_bytes(op.dtype));
    if (cnt == 1 && low == 0 && (int64_t(1) << pb) * 2 <= p.blocks && p.blocks >= 16 &&
        (tile_bytes << pb) >= kPairOrderMinBytes)
      p.map.pair_bit = pb;
  }
  if (p.map.run_log2 == 0 && p.map.pair_bit == 0) p.map.order = t.spmv_order;
  return p;
}

template <typename R, int RPT, int G, bool CHK, int KC, bool NT, bool DM>
void launch_one(diaq_ctx* ctx, const DiagArgs& da, const DiagSrc& src, const Plan& p,
                const typename Vec<R>::V* v, const typename Vec<R>::V* x, typename Vec<R>::V* y,
                double2* partial, const typename Vec<R>::V* psi) {
  dim3 grid(unsigned(p.blocks)), block(kBlock);
  if constexpr (!std::is_same<R, Pk>::value) {
    if (partial) {
      hipLaunchKernelGGL((expect_kernel<R, RPT, G, CHK, KC, false, DM>), grid, block, 0, ctx->stream, da, src, p.map,
                         v, psi, x, partial);
      return;
    }
  }
  hipLaunchKernelGGL((spmv_kernel<R, RPT, G, CHK, KC, NT, DM>), grid, block, 0, ctx->stream, da, src, p.map, v, x, y);
}

template <typename R, int RPT, int G, bool CHK>
void launch_kc(diaq_ctx* ctx, const DiagArgs& da, const DiagSrc& src, const Plan& p,
               const typename Vec<R>::V* v, const typename Vec<R>::V* x, typename Vec<R>::V* y, double2* partial,
               const typename Vec<R>::V* psi) {
  if (p.kc == 3) {
    if (p.nt) launch_one<R, RPT, G, CHK, 3, true, false>(ctx, da, src, p, v, x, y, partial, psi);
    else launch_one<R, RPT, G, CHK, 3, false, false>(ctx, da, src, p, v, x, y, partial, psi);
  } else {
    if (p.nt) launch_one<R, RPT, G, CHK, 1, true, false>(ctx, da, src, p, v, x, y, partial, psi);
    else launch_one<R, RPT, G, CHK, 1, false, false>(ctx, da, src, p, v, x, y, partial, psi);
  }
}

template <typename R>
diaq_status_t launch_typed(diaq_ctx* ctx, const SpmvOp& op, const DiagArgs& da, const DiagSrc& src,
                           const Plan& p, const void* vals, const void* x, void* y, double2* partial,
                           const void* psi) {
  using V = typename Vec<R>::V;
  const V* v = static_cast<const V*>(vals);
  const V* xx = static_cast<const V*>(x);
  V* yy = static_cast<V*>(y);
  const V* pp = static_cast<const V*>(psi);
  const int rows = p.rpt * p.g;
  if (src.dmeta) {
    // many diagonals: device descriptor table, no tile grouping
    if (p.check) launch_one<R, 1, 1, true, 3, false, true>(ctx, da, src, p, v, xx, yy, partial, pp);
    else if (p.nt) launch_one<R, 2, 1, false, 3, true, true>(ctx, da, src, p, v, xx, yy, partial, pp);
    else launch_one<R, 2, 1, false, 3, false, true>(ctx, da, src, p, v, xx, yy, partial, pp);
  } else if (p.check) launch_kc<R, 1, 1, true>(ctx, da, src, p, v, xx, yy, partial, pp);
  else if (p.g == 1 && p.rpt == 4) launch_kc<R, 4, 1, false>(ctx, da, src, p, v, xx, yy, partial, pp);
  else if (p.g == 1 && p.rpt == 2) launch_kc<R, 2, 1, false>(ctx, da, src, p, v, xx, yy, partial, pp);
  else if (p.g == 1) launch_kc<R, 1, 1, false>(ctx, da, src, p, v, xx, yy, partial, pp);
  else if (p.g == 2 && p.rpt == 2) launch_kc<R, 2, 2, false>(ctx, da, src, p, v, xx, yy, partial, pp);
  else if (p.g == 2) launch_kc<R, 1, 2, false>(ctx, da, src, p, v, xx, yy, partial, pp);
  else if (p.g == 4) launch_kc<R, 1, 4, false>(ctx, da, src, p, v, xx, yy, partial, pp);
  else if (p.g == 8 && rows == 8) launch_one<R, 1, 8, false, 1, false, false>(ctx, da, src, p, v, xx, yy, partial, pp);
  else return fail(DIAQ_ERR_DEVICE, "no SpMV variant for rows %d group %d", p.rpt, p.g);
  DIAQ_HIP(hipGetLastError());
  return DIAQ_OK;
}

diaq_status_t prepare(const SpmvOp& op, DiagArgs& da, DiagSrc& src) {
  std::memset(&da, 0, sizeof(da));
  src.nd = op.nd;
  src.transpose = op.transpose ? 1 : 0;
  src.conjugate = op.conjugate ? 1 : 0;
  src.skip_zero = op.skip_zero ? 1 : 0;
  if (op.nd <= kMaxArgDiags) {
    src.dmeta = nullptr;
    da.nd = op.nd;
    for (int k = 0; k < op.nd; k++) {
      da.off[k] = op.host_off[k];
      da.start[k] = op.host_start[k];
    }
  } else {
    if (!op.dmeta) return fail(DIAQ_ERR_INVALID_ARGUMENT, "matrix with %d diagonals has no device table", op.nd);
    src.dmeta = op.dmeta;
    da.nd = 0;
  }
  return DIAQ_OK;
}

// complex64 products that run packed (two amplitudes per 16-byte unit):
// every offset and diagonal start even, descriptors in the kernel
// arguments, 16-byte aligned vectors, and the knob not off.
bool packable(const SpmvOp& op, const diaq_tuning_t& t, const void* x, const void* y) {
  if (op.dtype != DIAQ_C64 || t.spmv_pack < 0 || op.n < 2 || op.nd > kMaxArgDiags) return false;
  for (int k = 0; k < op.nd; k++)
    if ((op.host_off[k] & 1) || (op.host_start[k] & 1)) return false;
  auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  return aligned(x) && aligned(y) && aligned(op.values);
}

// The packed problem: 2^(n-1) units, offsets and starts halved, coupling
// qubits one lower (qubit q of the state is bit q - 1 of a unit index), and
// the tile-pairing knobs moved down with them.
struct PackedOp {
  SpmvOp op;
  int64_t off[kMaxArgDiags], start[kMaxArgDiags];
  diaq_tuning_t t;
};
void pack_op(const SpmvOp& op, const diaq_tuning_t& t, PackedOp* P) {
  P->op = op;
  P->op.n = op.n - 1;
  P->op.dtype = DIAQ_C128;  // planned as 16-byte elements
  for (int k = 0; k < op.nd; k++) {
    P->off[k] = op.host_off[k] / 2;
    P->start[k] = op.host_start[k] / 2;
  }
  P->op.host_off = P->off;
  P->op.host_start = P->start;
  P->op.qubit_mask = op.qubit_mask >> 1;
  P->t = t;
  P->t.spmv_group_qubits = t.spmv_group_qubits >> 1;
  // (a threshold of qubit 1 stays 1: 0 would mean the default)
  P->t.spmv_group_min_qubit =
      std::max(1, (t.spmv_group_min_qubit > 0 ? t.spmv_group_min_qubit : kDefaultGroupMinQubit) - 1);
}

}  // namespace

diaq_status_t launch_spmv(diaq_ctx* ctx, const SpmvOp& op, const void* x, void* y) {
  const int64_t N = int64_t(1) << op.n;
  if (op.nd == 0) {
    DIAQ_HIP(hipMemsetAsync(y, 0, size_t(N) * elem_bytes(op.dtype), ctx->stream));
    return DIAQ_OK;
  }
  if (x == y) {
    // only a principal-diagonal-only matrix may run in place
    if (!(op.nd == 1 && op.host_off[0] == 0))
      return fail(DIAQ_ERR_INVALID_ARGUMENT, "x and y alias for a matrix with off-principal diagonals");
    const int64_t blocks = (N + kBlock - 1) / kBlock;  // one element per lane
    // complex128 streams with non-temporal hints (measured 5.76 -> 6.32
    // TB/s at n = 28), and so do complex64 pairs as 16-byte units (5.96 ->
    // 6.36 TB/s against one amplitude per lane; 5.72 without the hints);
    // single complex64 amplitudes are faster with plain accesses (5.95
    // against 5.03 TB/s)
    if (op.dtype == DIAQ_C128)
      hipLaunchKernelGGL((diag_inplace_kernel<double, true>), dim3(unsigned(blocks)), dim3(kBlock), 0, ctx->stream,
                         N, op.conjugate ? 1 : 0, static_cast<const double2*>(op.values), static_cast<double2*>(y));
    else if (packable(op, ctx->tuning, y, y))
      hipLaunchKernelGGL((diag_inplace_kernel<Pk, true>), dim3(unsigned((N / 2 + kBlock - 1) / kBlock)), dim3(kBlock),
                         0, ctx->stream, N / 2, op.conjugate ? 1 : 0, static_cast<const float4*>(op.values),
                         static_cast<float4*>(y));
    else
      hipLaunchKernelGGL((diag_inplace_kernel<float, false>), dim3(unsigned(blocks)), dim3(kBlock), 0, ctx->stream,
                         N, op.conjugate ? 1 : 0, static_cast<const float2*>(op.values), static_cast<float2*>(y));
    DIAQ_HIP(hipGetLastError());
    return DIAQ_OK;
  }
  DiagArgs da;
  DiagSrc src;
  if (packable(op, ctx->tuning, x, y)) {
    PackedOp P;
    pack_op(op, ctx->tuning, &P);
    DIAQ_TRY(prepare(P.op, da, src));
    const Plan p = plan_rows(P.op, P.t, ctx->spmv_rows);
    return launch_typed<Pk>(ctx, P.op, da, src, p, op.values, x, y, nullptr, nullptr);
  }
  DIAQ_TRY(prepare(op, da, src));
  const Plan p = plan_rows(op, ctx->tuning, ctx->spmv_rows);
  if (op.dtype == DIAQ_C128) return launch_typed<double>(ctx, op, da, src, p, op.values, x, y, nullptr, nullptr);
  return launch_typed<float>(ctx, op, da, src, p, op.values, x, y, nullptr, nullptr);
}

diaq_status_t spmv_shape(const SpmvOp& op, const diaq_tuning_t& t, diaq_spmv_shape_t* out) {
  std::memset(out, 0, sizeof(*out));
  for (int b = 0; b < 3; b++) out->group_qubits[b] = -1;
  const int64_t N = int64_t(1) << op.n;
  // (aligned vectors assumed: the library's own allocations are)
  static const char aligned_probe[16] __attribute__((aligned(16))) = {};
  const bool packed = packable(op, t, aligned_probe, aligned_probe);
  out->packed = packed ? 1 : 0;
  if (op.nd == 1 && op.host_off[0] == 0) {
    out->in_place = 1;
    out->rows_per_lane = 1;
    out->group = 1;
    out->chunk = 1;
    out->nontemporal = (op.dtype == DIAQ_C128 || packed) ? 1 : 0;
    out->tile_log2 = packed ? 9 : 8;
    out->blocks = ((packed ? N / 2 : N) + kBlock - 1) / kBlock;
    return DIAQ_OK;
  }
  PackedOp P;
  if (packed) pack_op(op, t, &P);
  const Plan p = packed ? plan_rows(P.op, P.t, 0) : plan_rows(op, t, 0);
  // the variant launch_typed instantiates for this plan
  out->rows_per_lane = p.rpt;
  out->group = p.g;
  if (op.nd > kMaxArgDiags) {
    out->chunk = 3;
    out->nontemporal = (!p.check && p.nt) ? 1 : 0;
  } else if (p.g == 8) {
    out->chunk = 1;
    out->nontemporal = 0;
  } else {
    out->chunk = p.kc;
    out->nontemporal = p.nt ? 1 : 0;
  }
  // packed units: a tile of 2^t units holds 2^(t+1) amplitudes, unit bit b
  // is qubit b + 1
  out->tile_log2 = p.map.tile_log2 + (packed ? 1 : 0);
  for (int b = 0; b < p.map.ng; b++) out->group_qubits[b] = p.map.gbit[b] + (packed ? 1 : 0);
  out->xcd_run_log2 = p.map.run_log2;
  out->pair_bit = p.map.pair_bit;
  out->tile_order = p.map.order;
  out->blocks = p.blocks;
  return DIAQ_OK;
}

diaq_status_t launch_final_reduce(hipStream_t stream, const double2* partial, int64_t count, double* dres) {
  hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(1024), 0, stream, partial, count,
                     reinterpret_cast<double2*>(dres));
  DIAQ_HIP(hipGetLastError());
  return DIAQ_OK;
}

static diaq_status_t final_reduce(diaq_ctx* ctx, const double2* partial, int64_t count, double* dres) {
  return launch_final_reduce(ctx->stream, partial, count, dres);
}

diaq_status_t launch_expect(diaq_ctx* ctx, const SpmvOp& op, const void* psi, const void* phi, double* dres) {
  if (op.nd == 0) {
    DIAQ_HIP(hipMemsetAsync(dres, 0, 2 * sizeof(double), ctx->stream));
    return DIAQ_OK;
  }
  DiagArgs da;
  DiagSrc src;
  DIAQ_TRY(prepare(op, da, src));
  const Plan p = plan_rows(op, ctx->tuning, ctx->spmv_rows);
  DIAQ_TRY(ensure(ctx, &ctx->red, size_t(p.blocks) * sizeof(double2)));
  double2* partial = static_cast<double2*>(ctx->red.ptr);
  if (op.dtype == DIAQ_C128)
    DIAQ_TRY(launch_typed<double>(ctx, op, da, src, p, op.values, phi, nullptr, partial, psi));
  else
    DIAQ_TRY(launch_typed<float>(ctx, op, da, src, p, op.values, phi, nullptr, partial, psi));
  return final_reduce(ctx, partial, p.blocks, dres);
}

namespace {
std::mutex g_static_mu;
double2* g_static_ptr[kMaxStaticDevices] = {};
}  // namespace

diaq_status_t init_static_scratch(int device) {
  if (device < 0 || device >= kMaxStaticDevices)
    return fail(DIAQ_ERR_UNSUPPORTED, "device %d beyond the %d devices of the static scratch table", device,
                kMaxStaticDevices);
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (g_static_ptr[device]) return DIAQ_OK;
  void* ptr = nullptr;
  DIAQ_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(DIAQ_ERR_DEVICE, "no device address for the static scratch of device %d", device);
  g_static_ptr[device] = static_cast<double2*>(ptr);
  return DIAQ_OK;
}

diaq_status_t launch_expect_static(diaq_ctx* ctx, const SpmvOp& op, const void* psi, const void* phi, double* dres) {
  double2* partial = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (ctx->device >= 0 && ctx->device < kMaxStaticDevices) partial = g_static_ptr[ctx->device];
  }
  if (!partial) return fail(DIAQ_ERR_DEVICE, "static scratch of device %d was not set up", ctx->device);
  // a matrix without diagonals: <psi|0|phi> = 0 by a fill kernel
  if (op.nd == 0) return launch_zero(ctx->stream, dres, 2 * sizeof(double));
  DiagArgs da;
  DiagSrc src;
  DIAQ_TRY(prepare(op, da, src));
  const Plan p = plan_rows(op, ctx->tuning, ctx->spmv_rows);
  if (p.blocks > kStaticPartials)
    return fail(DIAQ_ERR_UNSUPPORTED, "the product needs %lld partial sums, the static scratch holds %lld",
                (long long)p.blocks, (long long)kStaticPartials);
  // every workgroup writes its own partial, so nothing needs clearing
  if (op.dtype == DIAQ_C128)
    DIAQ_TRY(launch_typed<double>(ctx, op, da, src, p, op.values, phi, nullptr, partial, psi));
  else
    DIAQ_TRY(launch_typed<float>(ctx, op, da, src, p, op.values, phi, nullptr, partial, psi));
  return final_reduce(ctx, partial, p.blocks, dres);
}

diaq_status_t launch_generator_dot(diaq_ctx* ctx, const LocalGate& gen, int n, diaq_dtype_t dt,
                                   const void* lam, const void* psi, double* dres) {
  GenArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k = gen.k;
  a.ncos = (int64_t(1) << n) >> gen.k;
  for (int j = 0; j < gen.k; j++) a.tq[j] = gen.targets[j];
  int st[3] = {gen.targets[0], gen.targets[1], gen.targets[2]};
  std::sort(st, st + gen.k);
  for (int j = 0; j < gen.k; j++) a.sorted_t[j] = st[j];
  a.cmask = gen.cmask;
  std::memcpy(a.g, gen.m, sizeof(a.g));
  const int64_t blocks = (a.ncos + kBlock - 1) / kBlock;
  DIAQ_TRY(ensure(ctx, &ctx->red, size_t(blocks) * sizeof(double2)));
  double2* partial = static_cast<double2*>(ctx->red.ptr);
  if (dt == DIAQ_C128)
    hipLaunchKernelGGL(generator_dot_kernel<double>, dim3(unsigned(blocks)), dim3(kBlock), 0, ctx->stream, a,
                       static_cast<const double2*>(lam), static_cast<const double2*>(psi), partial);
  else
    hipLaunchKernelGGL(generator_dot_kernel<float>, dim3(unsigned(blocks)), dim3(kBlock), 0, ctx->stream, a,
                       static_cast<const float2*>(lam), static_cast<const float2*>(psi), partial);
  DIAQ_HIP(hipGetLastError());
  return final_reduce(ctx, partial, blocks, dres);
}

}  // namespace diaq

// kron.hip -- Alg. 3: y = (I_a (x) M (x) I_b) x without expanding the gate.
//
// Alg. 3 walks M's DiaQ diagonals and, for each, multiplies the diagonal's
// values into shifted subsets of x (offset dim_b * dIndex).  For targets
// that are not adjacent, or carry controls, the same product is organised
// by cosets: the amplitudes that differ only in the gate's target bits form
// a 2^k-vector v, and the gate maps it to M v (Alg. 3's rep and j loops
// enumerate these cosets for adjacent targets).  One lane owns whole cosets,
// so the product runs in place, reads and writes each amplitude once
// (2 N s bytes per gate, the minimum for a gate application) and needs no
// expanded diagonals and no scratch vector.  Diagonal gates are applied
// element-wise.  Diagonal gates folded in by the fusion planner multiply
// the output rows.
#include "internal.hpp"

namespace diaq {

namespace {

constexpr int kBlock = 256;
// One coset per lane and a full grid: in-place streams run faster with
// more workgroups in flight than with several cosets per lane.
constexpr int kCosetsPerLane = 1;

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

struct KronArgs {
  int64_t ncos;        // N >> k
  int64_t off[8];      // scatter(r): amplitude offset of local index r
  int32_t k;
  int32_t sorted[3];   // target qubits ascending (zero-bit insertion)
  uint64_t cmask;
  int32_t adjoint;
  int32_t nt;          // folded diagonal factors: tables at tabs
  int32_t rows;        // 1: the table headers hold this op's roff[r]
  int32_t ntio;        // 1: state loads and stores carry non-temporal hints
  int32_t order;       // workgroup order (kron_block)
  int32_t pack;        // complex64: two amplitudes per 16-byte access where possible
  const char* tabs;
  const double* dmat;  // device 4 x 4 local matrix (k <= 2), replaces m
  double m[8][8][2];
  double g[8][8][2];   // generator (adjoint step with a dot)
};

// Local matrix element (r, c), part j: from the kernel arguments, or with DM
// from device memory (matrices that depend on angles held on the device).
template <bool DM>
__device__ __forceinline__ double mel(const KronArgs& a, int r, int c, int j) {
  if constexpr (DM)
    return a.dmat[(r * 4 + c) * 2 + j];
  else
    return a.m[r][c][j];
}

// State accesses, non-temporal when nt (each amplitude is read and written
// once per operation).
template <typename V>
__device__ __forceinline__ V kld(const V* p, bool nt) {
  if (nt) {
    typedef decltype(V{}.x) E;
    typedef E N2 __attribute__((ext_vector_type(2)));
    const N2 t = __builtin_nontemporal_load(reinterpret_cast<const N2*>(p));
    return V{t[0], t[1]};
  }
  return *p;
}
template <typename V>
__device__ __forceinline__ void kst(V* p, const V& v, bool nt) {
  if (nt) {
    typedef decltype(V{}.x) E;
    typedef E N2 __attribute__((ext_vector_type(2)));
    N2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<N2*>(p));
  } else {
    *p = v;
  }
}

// The block of cosets workgroup b takes: launch order, each XCD (the
// device deals workgroups to its 8 XCDs in turn) a contiguous eighth of the
// blocks, or the two halves interleaved.
__device__ __forceinline__ int64_t kron_block(int order) {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  if (order == 1 && (nb & 7) == 0) return (b & 7) * (nb >> 3) + (b >> 3);
  if (order == 2 && (nb & 1) == 0) return (b >> 1) + (b & 1) * (nb >> 1);
  // 3: blocks scattered over the state (an odd multiplier permutes a
  // power-of-two count)
  if (order == 3 && (nb & (nb - 1)) == 0) return (b * 0x9E3779B1ll) & (nb - 1);
  return b;
}

__device__ __forceinline__ int64_t insert_zeros(int64_t v, const KronArgs& a) {
  for (int j = 0; j < a.k; j++) {
    const int p = a.sorted[j];
    v = (v & ((int64_t(1) << p) - 1)) | ((v >> p) << (p + 1));
  }
  return v;
}

template <int K, bool DM>
__device__ __forceinline__ void mat_vec(const KronArgs& a, const double (&xr)[1 << K], const double (&xi)[1 << K],
                                        double (&yr)[1 << K], double (&yi)[1 << K]) {
  constexpr int d = 1 << K;
#pragma unroll
  for (int r = 0; r < d; r++) {
    double sr = 0, si = 0;
#pragma unroll
    for (int c = 0; c < d; c++) {
      const double mr = a.adjoint ? mel<DM>(a, c, r, 0) : mel<DM>(a, r, c, 0);
      const double mi = a.adjoint ? -mel<DM>(a, c, r, 1) : mel<DM>(a, r, c, 1);
      sr += mr * xr[c] - mi * xi[c];
      si += mr * xi[c] + mi * xr[c];
    }
    yr[r] = sr;
    yi[r] = si;
  }
}

// In place: v <- (M or M^dagger) v on every coset whose controls are 1,
// then the folded diagonal factors.
// TAB: 1 factor tables (if any) looked up row by row, 2 tables whose
// headers hold the rows' index bits (one header decode per coset).
template <typename R, int K, bool DM, int TAB>
__global__ __launch_bounds__(kBlock) void kron_apply_kernel(KronArgs a, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  constexpr int d = 1 << K;
  const int64_t c0 = kron_block(a.order) * (kBlock * kCosetsPerLane) + threadIdx.x;
  int64_t base[kCosetsPerLane];
  bool ok[kCosetsPerLane];
  double xr[kCosetsPerLane][d], xi[kCosetsPerLane][d];
#pragma unroll
  for (int u = 0; u < kCosetsPerLane; u++) {
    const int64_t cb = c0 + u * kBlock;
    ok[u] = cb < a.ncos;
    base[u] = ok[u] ? insert_zeros(cb, a) : 0;
    ok[u] = ok[u] && ((uint64_t(base[u]) & a.cmask) == a.cmask);
#pragma unroll
    for (int r = 0; r < d; r++) {
      V t = ok[u] ? kld(v + base[u] + a.off[r], a.ntio != 0) : V{0, 0};
      xr[u][r] = double(t.x);
      xi[u][r] = double(t.y);
    }
  }
#pragma unroll
  for (int u = 0; u < kCosetsPerLane; u++) {
    if (!ok[u]) continue;
    double yr[d], yi[d];
    mat_vec<K, DM>(a, xr[u], xi[u], yr, yi);
    // (TAB 2 also keeps the row-by-row path behind a run-time test: with
    // both paths the compiler schedules the per-coset one in fewer
    // registers, 78 against 94 for eight rows)
    const bool rows = TAB == 2 && a.rows;
    if (a.nt && rows) apply_tables_rows<d>(a.tabs, a.nt, uint64_t(base[u]), yr, yi);
#pragma unroll
    for (int r = 0; r < d; r++) {
      if (a.nt && !rows) apply_tables(a.tabs, a.nt, uint64_t(base[u] + a.off[r]), yr[r], yi[r]);
      kst(v + base[u] + a.off[r], V{R(yr[r]), R(yi[r])}, a.ntio != 0);
    }
  }
  // rows whose controls are 0 keep their amplitude, but folded factors
  // still multiply them
  if (a.nt && a.cmask) {
#pragma unroll
    for (int u = 0; u < kCosetsPerLane; u++) {
      const int64_t cb = c0 + u * kBlock;
      if (cb >= a.ncos) continue;
      const int64_t b = insert_zeros(cb, a);
      if ((uint64_t(b) & a.cmask) == a.cmask) continue;
#pragma unroll
      for (int r = 0; r < d; r++) {
        V t = v[b + a.off[r]];
        double tr = double(t.x), ti = double(t.y);
        apply_tables(a.tabs, a.nt, uint64_t(b + a.off[r]), tr, ti);
        v[b + a.off[r]] = V{R(tr), R(ti)};
      }
    }
  }
}

// Complex64 states, two cosets per lane: when qubit 0 is neither a target
// nor a control, cosets 2m and 2m + 1 sit at bases b and b + 1 and share
// their control bits, so each of their rows is one 16-byte access holding
// both (instead of two 8-byte ones; n = 28, mean over target qubits: U3
// 5.39 -> 5.73 TB/s, CX controlled by the top qubit 4.34 -> 5.06, groups
// of three qubits 4.14 -> 5.24).
template <int K, bool DM, int TAB>
__global__ __launch_bounds__(kBlock) void kron_apply2_kernel(KronArgs a, float4* __restrict__ v) {
  constexpr int d = 1 << K;
  typedef float F4 __attribute__((ext_vector_type(4)));
  const int64_t m = kron_block(a.order) * kBlock + threadIdx.x;
  if (2 * m >= a.ncos) return;
  const int64_t b = insert_zeros(2 * m, a);
  const bool on = (uint64_t(b) & a.cmask) == a.cmask;
  if (!on && a.nt == 0) return;
  const bool nt = a.ntio != 0;
  double xr0[d], xi0[d], xr1[d], xi1[d];
#pragma unroll
  for (int r = 0; r < d; r++) {
    const F4* p = reinterpret_cast<const F4*>(v) + (b + a.off[r]) / 2;
    const F4 t = nt ? __builtin_nontemporal_load(p) : *p;
    xr0[r] = t[0];
    xi0[r] = t[1];
    xr1[r] = t[2];
    xi1[r] = t[3];
  }
  if (!on) {
    // controls 0: the amplitudes stay, the folded factors still apply
#pragma unroll
    for (int r = 0; r < d; r++) {
      apply_tables(a.tabs, a.nt, uint64_t(b + a.off[r]), xr0[r], xi0[r]);
      apply_tables(a.tabs, a.nt, uint64_t(b + 1 + a.off[r]), xr1[r], xi1[r]);
      F4 o = {float(xr0[r]), float(xi0[r]), float(xr1[r]), float(xi1[r])};
      F4* p = reinterpret_cast<F4*>(v) + (b + a.off[r]) / 2;
      if (nt) __builtin_nontemporal_store(o, p);
      else *p = o;
    }
    return;
  }
  double yr0[d], yi0[d], yr1[d], yi1[d];
  mat_vec<K, DM>(a, xr0, xi0, yr0, yi0);
  mat_vec<K, DM>(a, xr1, xi1, yr1, yi1);
  const bool rows = TAB == 2 && a.rows;
  if (a.nt && rows) {
    apply_tables_rows<d>(a.tabs, a.nt, uint64_t(b), yr0, yi0);
    apply_tables_rows<d>(a.tabs, a.nt, uint64_t(b + 1), yr1, yi1);
  }
#pragma unroll
  for (int r = 0; r < d; r++) {
    if (a.nt && !rows) {
      apply_tables(a.tabs, a.nt, uint64_t(b + a.off[r]), yr0[r], yi0[r]);
      apply_tables(a.tabs, a.nt, uint64_t(b + 1 + a.off[r]), yr1[r], yi1[r]);
    }
    F4 o = {float(yr0[r]), float(yi0[r]), float(yr1[r]), float(yi1[r])};
    F4* p = reinterpret_cast<F4*>(v) + (b + a.off[r]) / 2;
    if (nt) __builtin_nontemporal_store(o, p);
    else *p = o;
  }
}

// One amplitude of a diagonal gate: row i's phase (if its controls are 1)
// and the folded factors.
template <bool DM>
__device__ __forceinline__ void diag_one(const KronArgs& a, int64_t i, double& tr, double& ti) {
  if ((uint64_t(i) & a.cmask) == a.cmask) {
    int r = 0;
    for (int j = 0; j < a.k; j++)
      if ((i & a.off[1 << j]) != 0) r |= 1 << j;
    const double mr = mel<DM>(a, r, r, 0), mi = a.adjoint ? -mel<DM>(a, r, r, 1) : mel<DM>(a, r, r, 1);
    const double nr = mr * tr - mi * ti;
    ti = mr * ti + mi * tr;
    tr = nr;
  }
  if (a.nt) apply_tables(a.tabs, a.nt, uint64_t(i), tr, ti);
}

// Diagonal gates: element-wise phase, in place.
template <typename R, bool DM>
__global__ __launch_bounds__(kBlock) void kron_diag_kernel(KronArgs a, int64_t N, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += stride) {
    const bool on = (uint64_t(i) & a.cmask) == a.cmask;
    if (!on && a.nt == 0) continue;  // an unfolded controlled phase leaves these rows alone
    V t = kld(v + i, a.ntio != 0);
    double tr = double(t.x), ti = double(t.y);
    diag_one<DM>(a, i, tr, ti);
    kst(v + i, V{R(tr), R(ti)}, a.ntio != 0);
  }
}

// The same for complex64 states taken two amplitudes at a time (16-byte
// accesses, non-temporal: n = 28, diagonal gates 4.8 -> 5.8 TB/s against
// one 8-byte amplitude per lane, CZ 2.2 -> 3.1 on its half-state model).  A unit whose two rows both keep their
// amplitude is left alone; otherwise both are rewritten.
template <bool DM>
__global__ __launch_bounds__(kBlock) void kron_diag2_kernel(KronArgs a, int64_t units, float4* __restrict__ v) {
  typedef float F4 __attribute__((ext_vector_type(4)));
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t u = int64_t(blockIdx.x) * kBlock + threadIdx.x; u < units; u += stride) {
    const int64_t i = 2 * u;
    const bool on0 = (uint64_t(i) & a.cmask) == a.cmask, on1 = (uint64_t(i + 1) & a.cmask) == a.cmask;
    if (!on0 && !on1 && a.nt == 0) continue;
    const F4 t = __builtin_nontemporal_load(reinterpret_cast<const F4*>(v + u));
    double r0 = t[0], i0 = t[1], r1 = t[2], i1 = t[3];
    diag_one<DM>(a, i, r0, i0);
    diag_one<DM>(a, i + 1, r1, i1);
    F4 o = {float(r0), float(i0), float(r1), float(i1)};
    __builtin_nontemporal_store(o, reinterpret_cast<F4*>(v + u));
  }
}

// Adjoint step: per coset, the generator dot conj(lam) (G psi) on the
// current vectors (GEN), then psi <- U^dagger psi and lam <- U^dagger lam.
// One partial sum per workgroup.
template <typename R, int K, bool GEN, bool DM>
__global__ __launch_bounds__(kBlock) void kron_adjoint_kernel(KronArgs a, typename Vec<R>::V* __restrict__ psi,
                                                              typename Vec<R>::V* __restrict__ lam,
                                                              double2* __restrict__ partial, int32_t step_back) {
  using V = typename Vec<R>::V;
  constexpr int d = 1 << K;
  double dre = 0, dim = 0;
  const int64_t c0 = int64_t(blockIdx.x) * (kBlock * kCosetsPerLane) + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kCosetsPerLane; u++) {
    const int64_t cb = c0 + u * kBlock;
    if (cb >= a.ncos) continue;
    const int64_t b = insert_zeros(cb, a);
    if ((uint64_t(b) & a.cmask) != a.cmask) continue;
    double pr[d], pi[d], lr[d], li[d];
#pragma unroll
    for (int r = 0; r < d; r++) {
      const V p = psi[b + a.off[r]];
      const V l = lam[b + a.off[r]];
      pr[r] = double(p.x);
      pi[r] = double(p.y);
      lr[r] = double(l.x);
      li[r] = double(l.y);
    }
    if (GEN) {
#pragma unroll
      for (int r = 0; r < d; r++) {
        double gr = 0, gi = 0;
#pragma unroll
        for (int c = 0; c < d; c++) {
          gr += a.g[r][c][0] * pr[c] - a.g[r][c][1] * pi[c];
          gi += a.g[r][c][0] * pi[c] + a.g[r][c][1] * pr[c];
        }
        dre += lr[r] * gr + li[r] * gi;
        dim += lr[r] * gi - li[r] * gr;
      }
    }
    if (step_back) {
      double yr[d], yi[d];
      mat_vec<K, DM>(a, pr, pi, yr, yi);
#pragma unroll
      for (int r = 0; r < d; r++) psi[b + a.off[r]] = V{R(yr[r]), R(yi[r])};
      mat_vec<K, DM>(a, lr, li, yr, yi);
#pragma unroll
      for (int r = 0; r < d; r++) lam[b + a.off[r]] = V{R(yr[r]), R(yi[r])};
    }
  }
  if (GEN) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      dre += __shfl_xor(dre, off, 64);
      dim += __shfl_xor(dim, off, 64);
    }
    __shared__ double2 wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wsum[wave] = double2{dre, dim};
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
}

KronArgs make_args(const LocalGate& lg, int n, bool adjoint, const void* tabs, int nt) {
  KronArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k = lg.k;
  a.ncos = (int64_t(1) << n) >> lg.k;
  for (int r = 0; r < (1 << lg.k); r++) {
    int64_t o = 0;
    for (int j = 0; j < lg.k; j++)
      if ((r >> j) & 1) o |= int64_t(1) << lg.targets[j];
    a.off[r] = o;
  }
  int st[3] = {lg.targets[0], lg.targets[1], lg.targets[2]};
  std::sort(st, st + lg.k);
  for (int j = 0; j < lg.k; j++) a.sorted[j] = st[j];
  a.cmask = lg.cmask;
  a.adjoint = adjoint ? 1 : 0;
  a.tabs = static_cast<const char*>(tabs);
  a.nt = tabs ? nt : 0;
  std::memcpy(a.m, lg.m, sizeof(a.m));
  return a;
}

bool is_diagonal_local(const LocalGate& lg) {
  const int d = 1 << lg.k;
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++)
      if (r != c && lg.structural[r][c]) return false;
  return true;
}

// Per-coset header decoding pays off from this many tables (QFT-29 with
// 3-qubit groups, up to 10 tables per operation: 94 -> 84 ms); with fewer,
// its extra registers cost more than the scalar work it saves.
constexpr int kRowsMinTables = 3;

template <typename R, int K, bool DM>
void launch_apply_tab(const KronArgs& a, int tab, dim3 grid, dim3 block, hipStream_t stream,
                      typename Vec<R>::V* v) {
  if (tab == 2) hipLaunchKernelGGL((kron_apply_kernel<R, K, DM, 2>), grid, block, 0, stream, a, v);
  else hipLaunchKernelGGL((kron_apply_kernel<R, K, DM, 1>), grid, block, 0, stream, a, v);
}

template <int K, bool DM>
void launch_apply2_tab(const KronArgs& a, int tab, hipStream_t stream, void* v) {
  const dim3 grid(unsigned((a.ncos / 2 + kBlock - 1) / kBlock)), block(kBlock);
  if (tab == 2) hipLaunchKernelGGL((kron_apply2_kernel<K, DM, 2>), grid, block, 0, stream, a, static_cast<float4*>(v));
  else hipLaunchKernelGGL((kron_apply2_kernel<K, DM, 1>), grid, block, 0, stream, a, static_cast<float4*>(v));
}

template <typename R, bool DM>
void dispatch_apply(const KronArgs& a, int k, bool diag, int64_t N, int num_cus, hipStream_t stream, void* v) {
  using V = typename Vec<R>::V;
  if (diag) {
    const int64_t blocks = (N + kBlock - 1) / kBlock;
    if constexpr (std::is_same<R, float>::value) {
      if (a.pack && (reinterpret_cast<uintptr_t>(v) & 15) == 0 && N >= 2) {
        const int64_t units = N / 2;
        hipLaunchKernelGGL((kron_diag2_kernel<DM>), dim3(static_cast<unsigned>((units + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, stream, a, units, static_cast<float4*>(v));
        return;
      }
    }
    hipLaunchKernelGGL((kron_diag_kernel<R, DM>), dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, stream, a, N,
                       static_cast<V*>(v));
    return;
  }
  const int64_t blocks = (a.ncos + kBlock * kCosetsPerLane - 1) / (kBlock * kCosetsPerLane);
  const dim3 grid(static_cast<unsigned>(blocks)), block(kBlock);
  const int tab = (a.rows && a.nt >= kRowsMinTables) ? 2 : 1;
  if constexpr (std::is_same<R, float>::value) {
    // qubit 0 outside the gate: two cosets per lane, 16-byte accesses
    if (a.pack && a.sorted[0] >= 1 && (a.cmask & 1) == 0 && a.ncos >= 2 &&
        (reinterpret_cast<uintptr_t>(v) & 15) == 0) {
      if (k == 1) launch_apply2_tab<1, DM>(a, tab, stream, v);
      else if (k == 2) launch_apply2_tab<2, DM>(a, tab, stream, v);
      else if constexpr (!DM) launch_apply2_tab<3, false>(a, tab, stream, v);
      return;
    }
  }
  if (k == 1)
    launch_apply_tab<R, 1, DM>(a, tab, grid, block, stream, static_cast<V*>(v));
  else if (k == 2)
    launch_apply_tab<R, 2, DM>(a, tab, grid, block, stream, static_cast<V*>(v));
  else if constexpr (!DM)
    launch_apply_tab<R, 3, false>(a, tab, grid, block, stream, static_cast<V*>(v));
}

template <typename R, bool GEN, bool DM>
void dispatch_adjoint(const KronArgs& a, int k, int64_t blocks, hipStream_t stream, void* psi, void* lam,
                      double2* partial, int sb) {
  using V = typename Vec<R>::V;
  const dim3 grid(static_cast<unsigned>(blocks)), block(kBlock);
  if (k == 1)
    hipLaunchKernelGGL((kron_adjoint_kernel<R, 1, GEN, DM>), grid, block, 0, stream, a, static_cast<V*>(psi),
                       static_cast<V*>(lam), partial, sb);
  else if (k == 2)
    hipLaunchKernelGGL((kron_adjoint_kernel<R, 2, GEN, DM>), grid, block, 0, stream, a, static_cast<V*>(psi),
                       static_cast<V*>(lam), partial, sb);
  else if constexpr (!DM)
    hipLaunchKernelGGL((kron_adjoint_kernel<R, 3, GEN, false>), grid, block, 0, stream, a, static_cast<V*>(psi),
                       static_cast<V*>(lam), partial, sb);
}

}  // namespace

double kron_op_bytes(const LocalGate& core, int nf, int n, diaq_dtype_t dt) {
  const double full = 2.0 * double(elem_bytes(dt)) * double(int64_t(1) << n);
  return nf ? full : full / double(int64_t(1) << core.nc);
}

void kron_row_offsets(const LocalGate& lg, int64_t* off) {
  for (int r = 0; r < (1 << lg.k); r++) {
    int64_t o = 0;
    for (int j = 0; j < lg.k; j++)
      if ((r >> j) & 1) o |= int64_t(1) << lg.targets[j];
    off[r] = o;
  }
}

diaq_status_t launch_kron_apply(diaq_ctx* ctx, hipStream_t stream, const LocalGate& lg, int n, diaq_dtype_t dt,
                                void* v, bool adjoint, const void* tabs, int nt, const double* dmat, bool rows) {
  if (dmat && lg.k > 2) return fail(DIAQ_ERR_UNSUPPORTED, "device matrices cover at most 2 targets");
  KronArgs a = make_args(lg, n, adjoint, tabs, nt);
  a.dmat = dmat;
  a.rows = rows ? 1 : 0;
  // non-temporal state streams (complex128; measured at n = 28: U3 5.65 ->
  // 6.06 TB/s mean over the target qubits, diagonal gates 5.98 -> 6.31) when
  // every row of a cache line is rewritten: a control below the line size
  // without factor tables leaves every other row untouched, and such
  // partial lines stream slower with the hints (CZ with control 0: 2.76 ->
  // 2.14 TB/s); complex64 streams measured faster without
  const uint64_t line_rows = dt == DIAQ_C128 ? 7 : 15;
  const bool full_lines = (lg.cmask & line_rows) == 0 || nt > 0;
  const int knob = ctx->tuning.kron_nontemporal;
  a.ntio = (knob > 0 || (knob == 0 && dt == DIAQ_C128)) && full_lines ? 1 : 0;
  // XCD-contiguous order (each XCD streams its own eighth of the state;
  // n = 28, U3 mean over qubits 8-27 6.04 -> 6.28 TB/s, qubits 20-22 5.5 ->
  // 5.8-6.3; the two halves interleaved 6.08, blocks scattered 5.09) for
  // operations that rewrite every row; a control without factor tables
  // leaves whole regions idle, which that order would put on half the XCDs
  // (CX controlled by the top qubit 5.25 -> 5.02)
  a.order = ctx->tuning.kron_order != 0 ? ctx->tuning.kron_order : ((lg.cmask == 0 || nt > 0) ? 1 : 0);
  a.pack = ctx->tuning.spmv_pack >= 0 ? 1 : 0;
  const int64_t N = int64_t(1) << n;
  const bool diag = is_diagonal_local(lg);
  if (dt == DIAQ_C128) {
    if (dmat) dispatch_apply<double, true>(a, lg.k, diag, N, ctx->num_cus, stream, v);
    else dispatch_apply<double, false>(a, lg.k, diag, N, ctx->num_cus, stream, v);
  } else {
    if (dmat) dispatch_apply<float, true>(a, lg.k, diag, N, ctx->num_cus, stream, v);
    else dispatch_apply<float, false>(a, lg.k, diag, N, ctx->num_cus, stream, v);
  }
  DIAQ_HIP(hipGetLastError());
  return DIAQ_OK;
}

int64_t kron_adjoint_blocks(const LocalGate& lg, int n) {
  const int64_t ncos = (int64_t(1) << n) >> lg.k;
  return (ncos + kBlock * kCosetsPerLane - 1) / (kBlock * kCosetsPerLane);
}

diaq_status_t launch_kron_adjoint(diaq_ctx* ctx, hipStream_t stream, const LocalGate& lg, const LocalGate* gen, int n,
                                  diaq_dtype_t dt, void* psi, void* lam, double2* partial, bool step_back,
                                  const double* dmat) {
  (void)ctx;
  if (dmat && lg.k > 2) return fail(DIAQ_ERR_UNSUPPORTED, "device matrices cover at most 2 targets");
  KronArgs a = make_args(lg, n, true, nullptr, 0);
  a.dmat = dmat;
  if (gen) std::memcpy(a.g, gen->m, sizeof(a.g));
  const int64_t blocks = kron_adjoint_blocks(lg, n);
  const int sb = step_back ? 1 : 0;
  if (dt == DIAQ_C128) {
    if (gen) {
      if (dmat) dispatch_adjoint<double, true, true>(a, lg.k, blocks, stream, psi, lam, partial, sb);
      else dispatch_adjoint<double, true, false>(a, lg.k, blocks, stream, psi, lam, partial, sb);
    } else {
      if (dmat) dispatch_adjoint<double, false, true>(a, lg.k, blocks, stream, psi, lam, partial, sb);
      else dispatch_adjoint<double, false, false>(a, lg.k, blocks, stream, psi, lam, partial, sb);
    }
  } else {
    if (gen) {
      if (dmat) dispatch_adjoint<float, true, true>(a, lg.k, blocks, stream, psi, lam, partial, sb);
      else dispatch_adjoint<float, true, false>(a, lg.k, blocks, stream, psi, lam, partial, sb);
    } else {
      if (dmat) dispatch_adjoint<float, false, true>(a, lg.k, blocks, stream, psi, lam, partial, sb);
      else dispatch_adjoint<float, false, false>(a, lg.k, blocks, stream, psi, lam, partial, sb);
    }
  }
  DIAQ_HIP(hipGetLastError());
  return DIAQ_OK;
}

}  // namespace diaq

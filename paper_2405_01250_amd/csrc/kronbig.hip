// kronbig.hip -- Alg. 3 with fused groups of up to five qubits.
//
// On the in-place (Alg. 3) path an operation costs one read and one write of
// the state whatever its matrix, so fusing more gates into fewer operations
// is pure gain as long as the arithmetic stays under the memory time.  The
// planner here groups gates the same way as the three-qubit planner (a gate
// joins the latest operation that shares a qubit, which it may move past
// because it commutes with everything after it) but lets a group span up to
// five qubits, multiplying the gates' embedded matrices into one dense
// 2^k x 2^k matrix (controls are qubits of the group).  Diagonal gates that
// do not fit stay row factors of an operation.  A lane owns one coset of the
// group (Alg. 3's cosets), keeps its 2^k amplitudes in registers, reads the
// matrix by scalar loads and writes each output row as soon as it is formed.
#include <complex>

#include "internal.hpp"

namespace diaq {

namespace {

using Cd = std::complex<double>;
constexpr int kBigBlock = 256;
constexpr int kBigMaxFactors = 64;

// Matrix of gate lg on the group qubits S (bit j of a local index is S[j]):
// P_ctrl (x) M + (1 - P_ctrl) (x) 1, identity on the group's other qubits.
std::vector<Cd> embed_gate(const LocalGate& lg, const int* S, int k) {
  const int D = 1 << k;
  auto pos = [&](int q) {
    for (int j = 0; j < k; j++)
      if (S[j] == q) return j;
    return -1;
  };
  int tpos[3], cpos[3];
  uint32_t tm = 0;
  for (int j = 0; j < lg.k; j++) {
    tpos[j] = pos(lg.targets[j]);
    tm |= 1u << tpos[j];
  }
  for (int j = 0; j < lg.nc; j++) cpos[j] = pos(lg.controls[j]);
  std::vector<Cd> E(size_t(D) * D, Cd(0, 0));
  for (int r = 0; r < D; r++)
    for (int c = 0; c < D; c++) {
      bool on = true;
      for (int j = 0; j < lg.nc; j++) on = on && ((c >> cpos[j]) & 1);
      if (!on) {
        if (r == c) E[size_t(r) * D + c] = 1.0;
        continue;
      }
      if ((uint32_t(r ^ c)) & ~tm) continue;
      int lr = 0, lc = 0;
      for (int j = 0; j < lg.k; j++) {
        lr |= ((r >> tpos[j]) & 1) << j;
        lc |= ((c >> tpos[j]) & 1) << j;
      }
      E[size_t(r) * D + c] = Cd(lg.m[lr][lc][0], lg.m[lr][lc][1]);
    }
  return E;
}

// The matrix M of an operation on qubits Sold, widened to the group S.
std::vector<Cd> widen(const std::vector<Cd>& M, const int* Sold, int kold, const int* S, int k) {
  const int D = 1 << k, Dold = 1 << kold;
  int p[5];
  uint32_t om = 0;
  for (int j = 0; j < kold; j++) {
    for (int t = 0; t < k; t++)
      if (S[t] == Sold[j]) p[j] = t;
    om |= 1u << p[j];
  }
  std::vector<Cd> W(size_t(D) * D, Cd(0, 0));
  for (int r = 0; r < D; r++)
    for (int c = 0; c < D; c++) {
      if ((uint32_t(r ^ c)) & ~om) continue;
      int lr = 0, lc = 0;
      for (int j = 0; j < kold; j++) {
        lr |= ((r >> p[j]) & 1) << j;
        lc |= ((c >> p[j]) & 1) << j;
      }
      W[size_t(r) * D + c] = M[size_t(lr) * Dold + lc];
    }
  return W;
}

std::vector<Cd> matmul(const std::vector<Cd>& A, const std::vector<Cd>& B, int D) {
  std::vector<Cd> C(size_t(D) * D, Cd(0, 0));
  for (int i = 0; i < D; i++)
    for (int m = 0; m < D; m++) {
      const Cd a = A[size_t(i) * D + m];
      if (a == Cd(0, 0)) continue;
      for (int j = 0; j < D; j++) C[size_t(i) * D + j] += a * B[size_t(m) * D + j];
    }
  return C;
}

int gate_qubit_list(const LocalGate& lg, int* q) {
  int u = 0;
  for (int j = 0; j < lg.k; j++) q[u++] = lg.targets[j];
  for (int j = 0; j < lg.nc; j++) q[u++] = lg.controls[j];
  return u;
}

bool diagonal_gate(const LocalGate& lg) {
  for (int r = 0; r < (1 << lg.k); r++)
    for (int c = 0; c < (1 << lg.k); c++)
      if (r != c && lg.structural[r][c]) return false;
  return true;
}

// Row factor of a diagonal gate on at most three qubits (targets, then
// controls): its diagonal on those qubits.
bool make_factor(const LocalGate& lg, DiagFactor* f) {
  int q[6];
  const int u = gate_qubit_list(lg, q);
  if (u > 3 || !diagonal_gate(lg)) return false;
  const std::vector<Cd> E = embed_gate(lg, q, u);
  std::memset(f, 0, sizeof(*f));
  f->k = u;
  for (int j = 0; j < u; j++) f->q[j] = q[j];
  for (int r = 0; r < (1 << u); r++) {
    f->v[r][0] = E[size_t(r) * (1 << u) + r].real();
    f->v[r][1] = E[size_t(r) * (1 << u) + r].imag();
  }
  return true;
}

struct BigArgs {
  int64_t ncos;
  int32_t nt;
  int32_t nt_io;     // non-temporal state streams
  int32_t sorted[5];
  int32_t pad2;
  int64_t off[32];  // global offset of local index r
  const double* mat;             // D x D, row-major, interleaved complex
  const char* tabs;              // factor tables applied to the output rows
};

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

// State loads and stores, with non-temporal hints when nt (each amplitude
// is read and written once per operation).
template <typename V>
__device__ __forceinline__ V bld(const V* p, bool nt) {
  if (nt) {
    typedef decltype(V{}.x) E;
    typedef E N2 __attribute__((ext_vector_type(2)));
    const N2 t = __builtin_nontemporal_load(reinterpret_cast<const N2*>(p));
    return V{t[0], t[1]};
  }
  return *p;
}
template <typename V>
__device__ __forceinline__ void bst(V* p, const V& v, bool nt) {
  if (nt) {
    typedef decltype(V{}.x) E;
    typedef E N2 __attribute__((ext_vector_type(2)));
    N2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<N2*>(p));
  } else {
    *p = v;
  }
}

template <typename R, int K>
__global__ __launch_bounds__(kBigBlock) void kron_big_kernel(BigArgs a, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  constexpr int D = 1 << K;
  // the matrix through the constant address space: every lane reads the
  // same entry at the same time, so these are scalar loads into SGPRs that
  // feed the FMAs directly (staging it in LDS made the LDS-to-register
  // traffic, 16 B per lane per entry, the limit: layered n = 28 with
  // 5-qubit groups 157 -> 150 ms, TFIM-28 313 -> 292 ms)
  typedef __attribute__((address_space(4))) const double GD;
  GD* mp = (GD*)(a.mat);
  const int64_t c = int64_t(blockIdx.x) * kBigBlock + threadIdx.x;
  if (c >= a.ncos) return;
  int64_t base = c;
#pragma unroll
  for (int j = 0; j < K; j++) {
    const int p = a.sorted[j];
    base = (base & ((int64_t(1) << p) - 1)) | ((base >> p) << (p + 1));
  }
  double xr[D], xi[D];
#pragma unroll
  for (int r = 0; r < D; r++) {
    const V t = bld(v + base + a.off[r], a.nt_io != 0);
    xr[r] = double(t.x);
    xi[r] = double(t.y);
  }
  // each output row is written as soon as it is formed: the inputs stay in
  // registers, so the in-place update is safe
#pragma unroll
  for (int r = 0; r < D; r++) {
    // four independent partial sums per component keep the FMA chains short
    double pr[4] = {0, 0, 0, 0}, pi[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < D; q++) {
      const double2 m = double2{mp[2 * (r * D + q)], mp[2 * (r * D + q) + 1]};
      pr[q & 3] = fma(m.x, xr[q], fma(-m.y, xi[q], pr[q & 3]));
      pi[q & 3] = fma(m.x, xi[q], fma(m.y, xr[q], pi[q & 3]));
    }
    double yr = (pr[0] + pr[1]) + (pr[2] + pr[3]);
    double yi = (pi[0] + pi[1]) + (pi[2] + pi[3]);
    const int64_t i = base + a.off[r];
    if (a.nt) apply_tables(a.tabs, a.nt, uint64_t(i), yr, yi);
    bst(v + i, V{R(yr), R(yi)}, a.nt_io != 0);
  }
}

// Groups that touch the lowest qubits.  With a target at bit 0..2 the lanes
// of the per-coset kernel above read amplitudes 2^(q_min+1) or more elements
// apart, so each load instruction touches up to 64 cache lines.  Here a
// wave owns 64 consecutive cosets, whose union is a set of contiguous runs
// of at least 64 amplitudes: the wave loads it coalesced into LDS, each lane
// then applies the matrix to its coset out of LDS (in place), and the wave
// stores the set back coalesced.
//
// Index space: P = the group's qubits plus the 6 lowest other qubits,
// ascending; bit j of a staging index e stands for element bit P[j].  The
// block index fills the element bits outside P.  Staging slot of e:
// e ^ ((e >> swz) & smask), which spreads the lanes' coset rows over the
// LDS banks (swz = staging bit of lane bit 0; no swizzle, smask = 0, when
// that is bit 0 and the lanes already sit in consecutive slots).
constexpr int kLdsLanes = 64;
constexpr int kLdsCosetBits = 6;
// A group of up to four qubits is staged when it has a qubit below 6 (the
// per-coset lanes of a gate on qubit 3..5 read every other 2^q-element run,
// two cache lines per 16-byte element load: U3 at n = 28 on qubits 3-5,
// 5.5 -> 6.1 TB/s staged; complex64 keeps qubits below 3, as its staged
// four-qubit groups measured slower: 3.9 against 4.9 TB/s on the per-coset
// path one qubit higher); a five-qubit group only when it holds qubit 0
// (its 32 x 32 product is close to the memory time, and the staged kernel,
// with fewer waves per CU, overlaps the two less well: measured 1.9 ms per
// n = 28 operation on the per-coset path against 3.3 ms staged for qubits
// 1-5, 2.9 against 2.8 for qubits 0-4).
constexpr int kLowQubit = 6, kLowQubit64 = 3;
inline bool staged(const int* q, int k, int low) { return k >= 1 && (k <= 4 ? q[0] < low : q[0] == 0); }
// block order of the staged and row-split group kernels (every row of a
// dense group is rewritten, so no region idles): by default the two halves
// of the blocks interleaved (n = 28, complex128, mean over positions: four
// qubits 5.96 -> 6.16 TB/s, worst position 3.9 -> 5.5 (groups across
// qubits 17-20); three qubits staged below qubit 6 5.5 -> 6.0; five qubits
// unchanged, 4.6; XCD eighths 5.98, scattered blocks 5.28)
inline int group_order(const diaq_tuning_t& t) { return t.kron_order == 0 ? 2 : t.kron_order; }

// the staging threshold of the knobs (kron_stage_qubit: 0 default, -1 never)
inline int stage_low(const diaq_tuning_t& t, diaq_dtype_t dt) {
  if (t.kron_stage_qubit == 0) return dt == DIAQ_C128 ? kLowQubit : kLowQubit64;
  return t.kron_stage_qubit < 0 ? 0 : t.kron_stage_qubit;
}

struct LdsArgs {
  int32_t npos;
  int32_t pos[11];      // P ascending
  int32_t nruns;
  int32_t run[11];      // staging bits -> element bits: first e bit | len << 8 | first element bit << 16
  int32_t swz;
  int32_t smask;
  int32_t nt;
  int32_t nt_io;     // non-temporal state streams
  int64_t lane_off[kLdsCosetBits];  // element offset of lane bit i
  int32_t lane_e[kLdsCosetBits];    // staging bit of lane bit i
  int32_t order;                    // block order (lds_block)
  int32_t eoff[32];     // staging offset of local index r
  int64_t roff[32];     // element offset of local index r
  int64_t joff[32];     // element offset of staging index 64 j
  const double* mat;
  const char* tabs;
};

__device__ __forceinline__ int64_t staging_to_element(const LdsArgs& a, int e) {
  int64_t off = 0;
  for (int r = 0; r < a.nruns; r++) {
    const uint32_t w = uint32_t(a.run[r]);
    const uint32_t src = w & 31u, len = (w >> 8) & 31u, dst = (w >> 16) & 63u;
    off |= int64_t((uint32_t(e) >> src) & ((1u << len) - 1u)) << dst;
  }
  return off;
}

__device__ __forceinline__ int slot(const LdsArgs& a, int e) { return e ^ ((e >> a.swz) & a.smask); }

// The block of 64 cosets workgroup b stages: launch order, or each XCD (the
// device deals workgroups to its 8 XCDs in turn) a contiguous eighth.
__device__ __forceinline__ int64_t lds_block(int order) {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  if (order == 1 && (nb & 7) == 0) return (b & 7) * (nb >> 3) + (b >> 3);
  if (order == 2 && (nb & 1) == 0) return (b >> 1) + (b & 1) * (nb >> 1);
  // 3: blocks scattered over the state (an odd multiplier permutes a
  // power-of-two count)
  if (order == 3 && (nb & (nb - 1)) == 0) return (b * 0x9E3779B1ll) & (nb - 1);
  return b;
}

// PARTS waves per block: wave p computes rows [p D / PARTS, (p + 1) D /
// PARTS) of every coset, so the block shares one staged matrix and a
// five-qubit group keeps enough waves per CU to overlap its arithmetic with
// the memory stream.
template <typename R, int K, int PARTS>
__global__ __launch_bounds__(kLdsLanes * PARTS) void kron_lds_kernel(LdsArgs a, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  constexpr int D = 1 << K;
  constexpr int E = kLdsLanes * D;
  constexpr int T = kLdsLanes * PARTS;  // lanes per block
  constexpr int L = D / PARTS;           // loads per lane, rows per lane
  __shared__ double2 sx[E];
  const int tid = threadIdx.x;
  // the matrix by scalar loads, as in kron_big_kernel: a wave's rows are
  // uniform (its part index, read while every lane is active)
  typedef __attribute__((address_space(4))) const double GD;
  GD* mp = (GD*)(a.mat);
  const int part = __builtin_amdgcn_readfirstlane(tid / kLdsLanes);
  int64_t base = lds_block(a.order);
  for (int j = 0; j < a.npos; j++) {
    const int p = a.pos[j];
    base = (base & ((int64_t(1) << p) - 1)) | ((base >> p) << (p + 1));
  }
  // coalesced load of the block's amplitudes (consecutive e are consecutive
  // elements within each run of at least 64), all loads in flight before
  // the first LDS write; e = tid + T j maps to the disjoint sum of the
  // element offsets of tid and of T j
  const int64_t tid_el = base + staging_to_element(a, tid);
  {
    V t[L];
#pragma unroll
    for (int j = 0; j < L; j++) t[j] = bld(v + tid_el + a.joff[j * PARTS], a.nt_io != 0);
#pragma unroll
    for (int j = 0; j < L; j++) sx[slot(a, tid + j * T)] = double2{double(t[j].x), double(t[j].y)};
  }
  __syncthreads();
  const int lane = tid & (kLdsLanes - 1);
  int el = 0;
  int64_t lo = 0;
#pragma unroll
  for (int i = 0; i < kLdsCosetBits; i++)
    if ((lane >> i) & 1) {
      el |= 1 << a.lane_e[i];
      lo |= a.lane_off[i];
    }
  double xr[D], xi[D];
#pragma unroll
  for (int r = 0; r < D; r++) {
    const double2 t = sx[slot(a, el + a.eoff[r])];
    xr[r] = t.x;
    xi[r] = t.y;
  }
  // the other waves still read this coset's inputs
  if (PARTS > 1) __syncthreads();
#pragma unroll
  for (int rr = 0; rr < L; rr++) {
    const int r = part * L + rr;
    double pr[4] = {0, 0, 0, 0}, pi[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < D; q++) {
      const double2 m = double2{mp[2 * (r * D + q)], mp[2 * (r * D + q) + 1]};
      pr[q & 3] = fma(m.x, xr[q], fma(-m.y, xi[q], pr[q & 3]));
      pi[q & 3] = fma(m.x, xi[q], fma(m.y, xr[q], pi[q & 3]));
    }
    double yr = (pr[0] + pr[1]) + (pr[2] + pr[3]);
    double yi = (pi[0] + pi[1]) + (pi[2] + pi[3]);
    if (a.nt) apply_tables(a.tabs, a.nt, uint64_t(base + lo + a.roff[r]), yr, yi);
    sx[slot(a, el + a.eoff[r])] = double2{yr, yi};
  }
  __syncthreads();
  {
    double2 t[L];
#pragma unroll
    for (int j = 0; j < L; j++) t[j] = sx[slot(a, tid + j * T)];
#pragma unroll
    for (int j = 0; j < L; j++) bst(v + tid_el + a.joff[j * PARTS], V{R(t[j].x), R(t[j].y)}, a.nt_io != 0);
  }
}

// Dense groups with the rows split over the waves of a block (factor tables
// compiled with the group's 2^K row offsets).  The block
// stages 64 cosets in LDS exactly as kron_lds_kernel does; wave p then forms
// rows [p L, (p + 1) L) of every coset, taking the coset's 2^K inputs out of
// LDS one at a time, so a lane holds only its L output rows (not the 2^K
// inputs) and the kernel needs few enough registers for five blocks of a
// five-qubit group per CU: while some blocks multiply, others stream.
// (The per-coset kernel keeps all 32 amplitudes of a five-qubit coset in
// registers, 211 VGPRs, two waves per SIMD, and its 4096 FMAs per coset
// barely overlap with its memory phase.)
// G3: the matrix is given as (Re, Im, Re + Im) per entry and each complex
// product takes three real FMAs instead of four (3072 instead of 4096 per
// five-qubit coset).
template <typename R, int K, int PARTS, bool G3>
__global__ __launch_bounds__(kLdsLanes * PARTS) void kron_split_kernel(LdsArgs a, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  constexpr int D = 1 << K;
  constexpr int E = kLdsLanes * D;
  constexpr int T = kLdsLanes * PARTS;  // lanes per block
  constexpr int L = D / PARTS;           // rows per lane, loads per lane
  __shared__ double2 sx[E];
  const int tid = threadIdx.x;
  typedef __attribute__((address_space(4))) const double GD;
  GD* mp = (GD*)(a.mat);
  const int part = __builtin_amdgcn_readfirstlane(tid / kLdsLanes);
  int64_t base = lds_block(a.order);
  for (int j = 0; j < a.npos; j++) {
    const int p = a.pos[j];
    base = (base & ((int64_t(1) << p) - 1)) | ((base >> p) << (p + 1));
  }
  const int64_t tid_el = base + staging_to_element(a, tid);
  {
    V t[L];
#pragma unroll
    for (int j = 0; j < L; j++) t[j] = bld(v + tid_el + a.joff[j * PARTS], a.nt_io != 0);
#pragma unroll
    for (int j = 0; j < L; j++) sx[slot(a, tid + j * T)] = double2{double(t[j].x), double(t[j].y)};
  }
  __syncthreads();
  const int lane = tid & (kLdsLanes - 1);
  int el = 0;
  int64_t lo = 0;
#pragma unroll
  for (int i = 0; i < kLdsCosetBits; i++)
    if ((lane >> i) & 1) {
      el |= 1 << a.lane_e[i];
      lo |= a.lane_off[i];
    }
  const int r0 = part * L;
  double ar[L], ai[L];
  if constexpr (G3) {
    // three real products per complex one (Gauss): with m = a + i b and
    // x = c + i d, Re = sum a c - sum b d and Im = sum (a + b)(c + d) -
    // sum a c - sum b d; the table holds (a, b, a + b) per entry
    double p1[L], p2[L], p3[L];
#pragma unroll
    for (int rr = 0; rr < L; rr++) p1[rr] = p2[rr] = p3[rr] = 0;
#pragma unroll 4
    for (int q = 0; q < D; q++) {
      const double2 t = sx[slot(a, el + a.eoff[q])];
      const double sum = t.x + t.y;
#pragma unroll
      for (int rr = 0; rr < L; rr++) {
        const int m = 3 * ((r0 + rr) * D + q);
        p1[rr] = fma(mp[m], t.x, p1[rr]);
        p2[rr] = fma(mp[m + 1], t.y, p2[rr]);
        p3[rr] = fma(mp[m + 2], sum, p3[rr]);
      }
    }
#pragma unroll
    for (int rr = 0; rr < L; rr++) {
      ar[rr] = p1[rr] - p2[rr];
      ai[rr] = p3[rr] - p1[rr] - p2[rr];
    }
  } else {
#pragma unroll
    for (int rr = 0; rr < L; rr++) ar[rr] = ai[rr] = 0;
    // column by column: one input out of LDS, then its L products
#pragma unroll 4
    for (int q = 0; q < D; q++) {
      const double2 t = sx[slot(a, el + a.eoff[q])];
#pragma unroll
      for (int rr = 0; rr < L; rr++) {
        const int m = 2 * ((r0 + rr) * D + q);
        const double mr = mp[m], mi = mp[m + 1];
        ar[rr] = fma(mr, t.x, fma(-mi, t.y, ar[rr]));
        ai[rr] = fma(mr, t.y, fma(mi, t.x, ai[rr]));
      }
    }
  }
  // every wave has read its inputs before any output overwrites them
  __syncthreads();
  // the table headers carry the index bits of the 2^K row offsets, so each
  // table is decoded once for the lane's L rows
  if (a.nt) apply_tables_rows<L>(a.tabs, a.nt, uint64_t(base + lo), ar, ai, r0);
#pragma unroll
  for (int rr = 0; rr < L; rr++) sx[slot(a, el + a.eoff[r0 + rr])] = double2{ar[rr], ai[rr]};
  __syncthreads();
  {
    double2 t[L];
#pragma unroll
    for (int j = 0; j < L; j++) t[j] = sx[slot(a, tid + j * T)];
#pragma unroll
    for (int j = 0; j < L; j++) bst(v + tid_el + a.joff[j * PARTS], V{R(t[j].x), R(t[j].y)}, a.nt_io != 0);
  }
}

// Dense groups on the fp64 matrix cores.  A group's 2^K x 2^K complex
// matrix M acts on [Re x; Im x] as the real 2D x 2D matrix
// [[Re M, -Im M], [Im M, Re M]] (D = 2^K), so applying it to 16 cosets at
// once is a real (2D x 2D) * (2D x 16) product: 2D / 16 row tiles of
// v_mfma_f64_16x16x4f64, each accumulated over 2D / 4 slices of depth 4.
// Lane l of a wave holds column l % 16 (one coset) at depth l / 16 of every
// operand, so it loads its coset's inputs 4 s + l / 16 (s < D / 4) straight
// from the state: real parts feed the first D / 4 slices, imaginary parts
// the last D / 4.  Accumulator register j of lane l holds row 4 j + l / 16
// of tile i (measured layout), so the lane ends up with the complete outputs
// 16 i + 4 j + l / 16 (j < 4) of its coset, which it writes back in place; a wave owns its
// 16 cosets, so every input is read before any output of the tile is
// written.  The real matrix sits in LDS in operand order (one 8-byte read
// per lane per product, conflict-free) and is loaded once per block;
// blocks stay resident and step through the tiles.  The arithmetic (4096
// FMAs per five-qubit coset) runs on the matrix cores, which leaves the
// vector unit to address and move the state (the per-coset vector kernel
// issues every FMA itself and spends 211 VGPRs on it).
typedef double MfmaAcc __attribute__((ext_vector_type(4)));
constexpr int kMfmaBlock = 256;

struct MfmaArgs {
  int64_t ntiles;      // cosets / 16
  int32_t nt;          // factor tables at tabs
  int32_t nt_io;       // non-temporal state streams
  int32_t sorted[5];   // group qubits ascending
  int32_t pad;
  int64_t off[32];     // element offset of local index r
  const double* lmat;  // real matrix in operand order, [(i S + s) 64 + lane] (fp32 values for kron_mfmap_kernel<float>)
  const char* tabs;
};

// HOLD: the matrix operands stay in registers across tiles (the compiler
// hoists the loop-invariant LDS reads: 128 VGPRs for a five-qubit group,
// two waves per SIMD); otherwise every tile re-reads them from LDS (an
// opaque per-tile offset keeps the reads in the loop, about 80 VGPRs).
template <typename R, int K, bool HOLD>
__global__ __launch_bounds__(kMfmaBlock) void kron_mfma_kernel(MfmaArgs a, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  constexpr int D = 1 << K;
  constexpr int RT = 2 * D / 16;  // row tiles
  constexpr int S = 2 * D / 4;    // slices of depth 4
  constexpr int NX = D / 4;       // complex inputs per lane
  __shared__ double sm[RT * S * 64];
  for (int e = threadIdx.x; e < RT * S * 64; e += kMfmaBlock) sm[e] = a.lmat[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t waves = int64_t(gridDim.x) * (kMfmaBlock / 64);
  for (int64_t t = int64_t(blockIdx.x) * (kMfmaBlock / 64) + (threadIdx.x >> 6); t < a.ntiles; t += waves) {
    int64_t base = t * 16 + col;
#pragma unroll
    for (int j = 0; j < K; j++) {
      const int p = a.sorted[j];
      base = (base & ((int64_t(1) << p) - 1)) | ((base >> p) << (p + 1));
    }
    double xr[NX], xi[NX];
#pragma unroll
    for (int s = 0; s < NX; s++) {
      const V x = bld(v + base + a.off[4 * s + kq], a.nt_io != 0);
      xr[s] = double(x.x);
      xi[s] = double(x.y);
    }
    MfmaAcc acc[RT];
#pragma unroll
    for (int i = 0; i < RT; i++) acc[i] = MfmaAcc{0, 0, 0, 0};
    int mo = lane;
    if constexpr (!HOLD) asm volatile("" : "+v"(mo));  // not loop-invariant: no hoisting
#pragma unroll
    for (int s = 0; s < S; s++) {
      const double b = s < NX ? xr[s] : xi[s - NX];
#pragma unroll
      for (int i = 0; i < RT; i++)
        acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(sm[(i * S + s) * 64 + mo], b, acc[i], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < RT / 2; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int r = 16 * i + 4 * j + kq;
        double yr = acc[i][j], yi = acc[i + RT / 2][j];
        const int64_t e = base + a.off[r];
        if (a.nt) apply_tables(a.tabs, a.nt, uint64_t(e), yr, yi);
        bst(v + e, V{R(yr), R(yi)}, a.nt_io != 0);
      }
  }
}

// The real form of the D x D complex matrix m (row-major, interleaved) in
// the operand order of kron_mfma_kernel: entry (i S + s) 64 + l holds
// row 16 i + l % 16, column 4 s + l / 16 of [[Re, -Im], [Im, Re]].
std::vector<double> mfma_operands(const std::vector<Cd>& m, int k) {
  const int D = 1 << k, RT = 2 * D / 16, S = 2 * D / 4;
  std::vector<double> out(size_t(RT) * S * 64);
  for (int i = 0; i < RT; i++)
    for (int s = 0; s < S; s++)
      for (int l = 0; l < 64; l++) {
        const int row = 16 * i + l % 16, c = 4 * s + l / 16;
        const Cd z = m[size_t(row % D) * D + (c % D)];
        double val;
        if (row < D) val = c < D ? z.real() : -z.imag();
        else val = c < D ? z.imag() : z.real();
        out[(size_t(i) * S + s) * 64 + l] = val;
      }
  return out;
}

// The operands of kron_mfmap_kernel's three products in operand order: entry
// ((p RT + i) S + s) 64 + l holds row 16 i + l % 16, column 4 s + l / 16 of
// Re M (p = 0), Im M (p = 1) or Re M + Im M (p = 2); RT = D / 16, S = D / 4.
std::vector<double> mfmap_operands(const std::vector<Cd>& m, int k) {
  const int D = 1 << k, RT = D / 16, S = D / 4;
  std::vector<double> out(size_t(3) * RT * S * 64);
  for (int p = 0; p < 3; p++)
    for (int i = 0; i < RT; i++)
      for (int s = 0; s < S; s++)
        for (int l = 0; l < 64; l++) {
          const Cd z = m[size_t(16 * i + l % 16) * D + (4 * s + l / 16)];
          out[((size_t(p) * RT + i) * S + s) * 64 + l] = p == 0 ? z.real() : p == 1 ? z.imag() : z.real() + z.imag();
        }
  return out;
}

// The matrix-core kernel needs 16 cosets of consecutive elements per tile
// (every group qubit >= 4) and at least one tile.
inline bool mfma_group(const int* q, int k, int n) { return (k == 4 || k == 5) && q[0] >= 4 && n >= k + 4; }

template <typename R>
void launch_mfma(const MfmaArgs& a, int k, bool hold, int num_cus, hipStream_t stream, void* state) {
  using V = typename Vec<R>::V;
  const int64_t want = (a.ntiles + 3) / 4;
  // resident blocks: four (16 waves) per CU, two when a five-qubit
  // group's matrix is held in registers
  const int64_t resident = int64_t(num_cus) * ((hold && k == 5) ? 2 : 4);
  const dim3 grid(unsigned(std::max<int64_t>(1, std::min(want, resident)))), block(kMfmaBlock);
  V* v = static_cast<V*>(state);
  if (k == 4) hipLaunchKernelGGL((kron_mfma_kernel<R, 4, true>), grid, block, 0, stream, a, v);
  else if (hold) hipLaunchKernelGGL((kron_mfma_kernel<R, 5, true>), grid, block, 0, stream, a, v);
  else hipLaunchKernelGGL((kron_mfma_kernel<R, 5, false>), grid, block, 0, stream, a, v);
}

// Pipelined matrix-core groups: the group's D x D complex matrix applied to
// 16 cosets at a time on the matrix cores (a tile: lane l holds column
// l % 16, one coset, at depth l / 16 of every operand, as in
// kron_mfma_kernel), arranged so that the memory stream and the matrix
// cores overlap.  Each wave loads the inputs of its next tile into a
// second register buffer before it multiplies the current one; the
// operand tables stay in LDS (a.lmat holds them in the state's precision),
// re-read for every tile, which leaves registers for three or more waves
// per SIMD; lane l's element offsets split into a wave-uniform part and a
// part fixed by l / 16, formed once, so the loop indexes no argument array
// by lane; the state is accessed without non-temporal hints, and factor
// tables are a separate instance (TAB): branches around the loads and
// stores make the compiler wait for every access, the prefetch included.
// Complex64 runs on the fp32 matrix cores (v_mfma_f32_16x16x4f32, operands
// and sums in fp32, the precision of its amplitudes; the vector kernels
// widen them to fp64), whose 16x16x4 step takes half the cycles of the
// fp64 one, so a five-qubit group's products fit under the memory time of
// its 8-byte amplitudes.  Complex128 runs on v_mfma_f64_16x16x4f64.
// Accumulator register j of lane l holds row 4 (l / 16) + j of its tile
// for fp32 and row 4 j + l / 16 for fp64 (both measured).
typedef float MfmaAcc32 __attribute__((ext_vector_type(4)));

template <typename R>
struct MfmaStep;
template <>
struct MfmaStep<float> {
  using Acc = MfmaAcc32;
  static constexpr bool kRowsByGroup = true;  // register j: row 4 (l / 16) + j
  static __device__ __forceinline__ Acc step(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaStep<double> {
  using Acc = MfmaAcc;
  static constexpr bool kRowsByGroup = false;  // register j: row 4 j + l / 16
  static __device__ __forceinline__ Acc step(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// The multiply-and-store of one tile whose inputs x (NX complex values of
// lane l's coset, local indices 4 s + l / 16) are in registers; dst is the
// tile's first element plus the lane's column and its output offset.  The
// complex product M v = (A + iB)(x + iy) takes three real D x D products
// instead of the four of the real 2D x 2D form: p1 = A x, p2 = B y,
// p3 = (A + B)(x + y), then Re = p1 - p2 and Im = p3 - p1 - p2 (48 instead
// of 64 matrix-core steps per five-qubit tile).
template <typename R, int K, bool TAB>
__device__ __forceinline__ void mfmap_tile(const MfmaArgs& a, typename Vec<R>::V* v, const R* sm, int mo,
                                           const typename Vec<R>::V (&x)[1 << (K - 2)], typename Vec<R>::V* dst) {
  using M = MfmaStep<R>;
  using V = typename Vec<R>::V;
  constexpr int D = 1 << K;
  constexpr int RT = D / 16;  // row tiles of each D x D product
  constexpr int S = D / 4;    // slices of depth 4
  typename M::Acc p1[RT], p2[RT], p3[RT];
#pragma unroll
  for (int i = 0; i < RT; i++) p1[i] = p2[i] = p3[i] = typename M::Acc{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < S; s++) {
    const R bx = x[s].x, by = x[s].y, bs = bx + by;
#pragma unroll
    for (int i = 0; i < RT; i++) {
      p1[i] = M::step(sm[((0 * RT + i) * S + s) * 64 + mo], bx, p1[i]);
      p2[i] = M::step(sm[((1 * RT + i) * S + s) * 64 + mo], by, p2[i]);
      p3[i] = M::step(sm[((2 * RT + i) * S + s) * 64 + mo], bs, p3[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < RT; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      R yr = p1[i][j] - p2[i][j], yi = p3[i][j] - p1[i][j] - p2[i][j];
      V* const o = dst + a.off[M::kRowsByGroup ? 16 * i + j : 16 * i + 4 * j];
      if constexpr (TAB) {
        double dr = yr, di = yi;
        apply_tables(a.tabs, a.nt, uint64_t(o - v), dr, di);
        yr = R(dr);
        yi = R(di);
      }
      *o = V{yr, yi};
    }
}

template <typename R, int K, bool TAB>
__global__ __launch_bounds__(kMfmaBlock) void kron_mfmap_kernel(MfmaArgs a, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  constexpr int D = 1 << K;
  constexpr int NX = D / 4;
  constexpr int TABN = 3 * (D / 16) * (D / 4) * 64;  // the three operand tables
  __shared__ R sm[TABN];
  const R* lm = reinterpret_cast<const R*>(a.lmat);
  for (int e = threadIdx.x; e < TABN; e += kMfmaBlock) sm[e] = lm[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  // off[] is additive over disjoint index bits: the lane's inputs are
  // local indices 4 s + kq, its outputs 16 i + 4 kq + j (fp32) or
  // 16 i + 4 j + kq (fp64)
  const int64_t in_lo = ((kq & 1) ? a.off[1] : 0) + ((kq & 2) ? a.off[2] : 0);
  const int64_t out_lane =
      MfmaStep<R>::kRowsByGroup ? ((kq & 1) ? a.off[4] : 0) + ((kq & 2) ? a.off[8] : 0) : in_lo;
  const int64_t waves = int64_t(gridDim.x) * (kMfmaBlock / 64);
  // a tile is 16 consecutive cosets; every group qubit is >= 4, so the
  // coset bits 0-3 (the lane's column) pass through unchanged and the
  // tile's first element is wave-uniform
  auto tile_first = [&](int64_t t) {
    int64_t b = t * 16;
#pragma unroll
    for (int j = 0; j < K; j++) {
      const int p = a.sorted[j];
      b = (b & ((int64_t(1) << p) - 1)) | ((b >> p) << (p + 1));
    }
    return b;
  };
  auto load = [&](V (&x)[NX], int64_t t) {
    const V* src = v + tile_first(t) + col + in_lo;
#pragma unroll
    for (int s = 0; s < NX; s++) x[s] = src[a.off[4 * s]];
  };
  int64_t t = int64_t(blockIdx.x) * (kMfmaBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (t >= a.ntiles) return;
  int mo = lane;
  // two input buffers in turn: while one tile is multiplied, the next
  // tile's loads are in flight into the other (the last tile's inputs are
  // loaded again past the end: in bounds, unused; tiles are disjoint, so a
  // tile's outputs are never among the inputs in flight)
  V xa[NX], xb[NX];
  load(xa, t);
  for (;;) {
    load(xb, std::min(t + waves, a.ntiles - 1));
    asm volatile("" : "+v"(mo));  // re-read the matrix for every tile (no hoisting)
    mfmap_tile<R, K, TAB>(a, v, sm, mo, xa, v + tile_first(t) + col + out_lane);
    t += waves;
    if (t >= a.ntiles) break;
    load(xa, std::min(t + waves, a.ntiles - 1));
    asm volatile("" : "+v"(mo));
    mfmap_tile<R, K, TAB>(a, v, sm, mo, xb, v + tile_first(t) + col + out_lane);
    t += waves;
    if (t >= a.ntiles) break;
  }
}

// resident blocks per CU of an instance, from its registers and LDS
template <typename R, int K, bool TAB>
int mfmap_resident() {
  static const int nb = [] {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kron_mfmap_kernel<R, K, TAB>, kMfmaBlock, 0) != hipSuccess) {
      (void)hipGetLastError();  // one block per CU, and no error left for the launch check
      b = 0;
    }
    return std::max(b, 1);
  }();
  return nb;
}

template <typename R, int K, bool TAB>
void launch_mfmap_k(const MfmaArgs& a, int num_cus, hipStream_t stream, void* state) {
  // persistent: as many blocks as stay resident together, so that no block
  // waits for another block's whole share of the tiles
  const int64_t want = (a.ntiles + 3) / 4;
  const int64_t resident = int64_t(num_cus) * mfmap_resident<R, K, TAB>();
  const dim3 grid(unsigned(std::max<int64_t>(1, std::min(want, resident)))), block(kMfmaBlock);
  hipLaunchKernelGGL((kron_mfmap_kernel<R, K, TAB>), grid, block, 0, stream, a,
                     static_cast<typename Vec<R>::V*>(state));
}

template <typename R>
void launch_mfmap(const MfmaArgs& a, int k, int num_cus, hipStream_t stream, void* state) {
  if (k == 4) {
    if (a.nt) launch_mfmap_k<R, 4, true>(a, num_cus, stream, state);
    else launch_mfmap_k<R, 4, false>(a, num_cus, stream, state);
  } else {
    if (a.nt) launch_mfmap_k<R, 5, true>(a, num_cus, stream, state);
    else launch_mfmap_k<R, 5, false>(a, num_cus, stream, state);
  }
}

// Staging layout for the group S (ascending) on n qubits; false if the
// state has fewer than 64 cosets.
bool make_lds_args(const int* S, int k, int n, LdsArgs* a) {
  if (n < k + kLdsCosetBits) return false;
  std::memset(a, 0, sizeof(*a));
  int P[11], np = 0, nl = 0;
  int lane_bits[kLdsCosetBits];
  for (int b = 0; b < n && np < k + kLdsCosetBits; b++) {
    bool in_s = false;
    for (int j = 0; j < k; j++) in_s = in_s || S[j] == b;
    if (!in_s && nl == kLdsCosetBits) continue;
    if (!in_s) lane_bits[nl++] = b;
    P[np++] = b;
  }
  a->npos = np;
  for (int j = 0; j < np; j++) a->pos[j] = P[j];
  auto eidx = [&](int b) {
    int j = 0;
    while (P[j] != b) j++;
    return j;
  };
  for (int i = 0; i < np;) {
    int e = i;
    while (e + 1 < np && P[e + 1] == P[e] + 1) e++;
    a->run[a->nruns++] = i | ((e - i + 1) << 8) | (P[i] << 16);
    i = e + 1;
  }
  for (int i = 0; i < kLdsCosetBits; i++) {
    a->lane_e[i] = eidx(lane_bits[i]);
    a->lane_off[i] = int64_t(1) << lane_bits[i];
  }
  a->swz = a->lane_e[0];
  a->smask = a->swz ? 15 : 0;
  for (int r = 0; r < (1 << k); r++) {
    int eo = 0;
    int64_t ro = 0;
    for (int j = 0; j < k; j++)
      if ((r >> j) & 1) {
        eo |= 1 << eidx(S[j]);
        ro |= int64_t(1) << S[j];
      }
    a->eoff[r] = eo;
    a->roff[r] = ro;
  }
  for (int j = 0; j < (1 << k); j++) {
    int64_t o = 0;
    for (int b = 0; b < k; b++)
      if ((j >> b) & 1) o |= int64_t(1) << P[kLdsCosetBits + b];
    a->joff[j] = o;
  }
  return true;
}

// rows = 8 or 4 output rows per wave (k = 4 or 5); g3: a.mat holds the
// (Re, Im, Re + Im) table of the three-multiplication product
template <typename R>
void launch_split(const LdsArgs& a, int k, int rows, bool g3, int n, hipStream_t stream, void* state) {
  using V = typename Vec<R>::V;
  const dim3 grid(unsigned((int64_t(1) << n) >> (k + kLdsCosetBits)));
  V* v = static_cast<V*>(state);
  if (k == 4 && rows == 8)
    hipLaunchKernelGGL((kron_split_kernel<R, 4, 2, false>), grid, dim3(kLdsLanes * 2), 0, stream, a, v);
  else if (k == 4)
    hipLaunchKernelGGL((kron_split_kernel<R, 4, 4, false>), grid, dim3(kLdsLanes * 4), 0, stream, a, v);
  else if (rows == 8 && g3)
    hipLaunchKernelGGL((kron_split_kernel<R, 5, 4, true>), grid, dim3(kLdsLanes * 4), 0, stream, a, v);
  else if (rows == 8)
    hipLaunchKernelGGL((kron_split_kernel<R, 5, 4, false>), grid, dim3(kLdsLanes * 4), 0, stream, a, v);
  else
    hipLaunchKernelGGL((kron_split_kernel<R, 5, 8, false>), grid, dim3(kLdsLanes * 8), 0, stream, a, v);
}

template <typename R>
void launch_lds(const LdsArgs& a, int k, int n, hipStream_t stream, void* state) {
  using V = typename Vec<R>::V;
  const dim3 grid(unsigned((int64_t(1) << n) >> (k + kLdsCosetBits)));
  const dim3 one(kLdsLanes), four(kLdsLanes * 4);
  V* v = static_cast<V*>(state);
  switch (k) {
    case 1: hipLaunchKernelGGL((kron_lds_kernel<R, 1, 1>), grid, one, 0, stream, a, v); break;
    case 2: hipLaunchKernelGGL((kron_lds_kernel<R, 2, 1>), grid, one, 0, stream, a, v); break;
    case 3: hipLaunchKernelGGL((kron_lds_kernel<R, 3, 1>), grid, one, 0, stream, a, v); break;
    case 4: hipLaunchKernelGGL((kron_lds_kernel<R, 4, 1>), grid, one, 0, stream, a, v); break;
    default: hipLaunchKernelGGL((kron_lds_kernel<R, 5, 4>), grid, four, 0, stream, a, v); break;
  }
}

}  // namespace

bool staged_dense(const LocalGate& lg, int n, int tables, const diaq_tuning_t& t, diaq_dtype_t dt,
                  std::vector<double>* mat, int* S, int* k) {
  // uncontrolled operations, or ones whose factors touch every row anyway
  // (a controlled one without them reads only its control-on half)
  if (lg.nc && !tables) return false;
  int q[6];
  const int u = gate_qubit_list(lg, q);
  if (u > 4) return false;
  std::sort(q, q + u);
  if (!staged(q, u, stage_low(t, dt))) return false;
  LdsArgs probe;
  if (!make_lds_args(q, u, n, &probe)) return false;
  const std::vector<Cd> E = embed_gate(lg, q, u);
  mat->resize(2 * E.size());
  for (size_t i = 0; i < E.size(); i++) {
    (*mat)[2 * i] = E[i].real();
    (*mat)[2 * i + 1] = E[i].imag();
  }
  for (int j = 0; j < u; j++) S[j] = q[j];
  *k = u;
  return true;
}

diaq_status_t launch_staged(diaq_ctx* ctx, const int* S, int k, const double* dmat, const char* tabs, int nt, int n,
                            diaq_dtype_t dt, void* state) {
  LdsArgs la;
  if (!make_lds_args(S, k, n, &la)) return fail(DIAQ_ERR_UNSUPPORTED, "staged group of %d qubits at n = %d", k, n);
  la.mat = dmat;
  la.tabs = tabs;
  la.nt = tabs ? nt : 0;
  la.order = group_order(ctx->tuning);
  la.nt_io = (k <= 4 && dt == DIAQ_C128) ? 1 : 0;
  if (dt == DIAQ_C128) launch_lds<double>(la, k, n, ctx->stream, state);
  else launch_lds<float>(la, k, n, ctx->stream, state);
  DIAQ_HIP(hipGetLastError());
  return DIAQ_OK;
}

namespace {

diaq_status_t plan_big_greedy(const diaq_gate_t* gates, int64_t ngates, int n, int kmax, std::vector<BigOp>* ops) {
  ops->clear();
  for (int64_t gi = 0; gi < ngates; gi++) {
    LocalGate lg;
    diaq_status_t st = local_gate(&gates[gi], n, &lg);
    if (st != DIAQ_OK) return fail(st, "gate %lld: %s", (long long)gi, diaq_last_error());
    int gq[6];
    const int gu = gate_qubit_list(lg, gq);
    uint64_t gm = 0;
    for (int j = 0; j < gu; j++) gm |= uint64_t(1) << gq[j];
    int64_t host = -1;
    for (int64_t k = int64_t(ops->size()) - 1; k >= 0; k--)
      if ((*ops)[k].mask & gm) {
        host = k;
        break;
      }
    DiagFactor f;
    const bool is_diag = make_factor(lg, &f);
    if (host >= 0) {
      BigOp& X = (*ops)[host];
      uint64_t fm = 0;
      for (const auto& pf : X.post)
        for (int j = 0; j < pf.k; j++) fm |= uint64_t(1) << pf.q[j];
      int S[8];
      int k = X.k;
      for (int j = 0; j < k; j++) S[j] = X.q[j];
      for (int j = 0; j < gu; j++) {
        bool seen = false;
        for (int t = 0; t < k; t++) seen = seen || S[t] == gq[j];
        if (!seen && k < 8) S[k++] = gq[j];
      }
      if (!X.raw && k <= kmax && (is_diag || !(fm & gm))) {
        std::sort(S, S + k);
        const std::vector<Cd> A = widen(X.m, X.q, X.k, S, k);
        const std::vector<Cd> B = embed_gate(lg, S, k);
        X.m = matmul(B, A, 1 << k);  // g after the operation
        X.k = k;
        for (int j = 0; j < k; j++) X.q[j] = S[j];
        X.mask |= gm;
        X.ngates++;
        continue;
      }
      if (is_diag && int(X.post.size()) < kBigMaxFactors) {
        X.post.push_back(f);
        X.mask |= gm;  // later gates on these qubits must not move before it
        X.ngates++;
        continue;
      }
    } else if (is_diag && !ops->empty() && int(ops->back().post.size()) < kBigMaxFactors) {
      ops->back().post.push_back(f);
      ops->back().mask |= gm;
      ops->back().ngates++;
      continue;
    }
    BigOp op;
    op.mask = gm;
    op.ngates = 1;
    if (gu > 5) {
      // more than five qubits with its controls: applied as it is
      op.raw = true;
      op.lg = lg;
      op.k = gu;
    } else {
      op.k = gu;
      for (int j = 0; j < gu; j++) op.q[j] = gq[j];
      std::sort(op.q, op.q + gu);
      op.m = embed_gate(lg, op.q, gu);
    }
    ops->push_back(std::move(op));
  }
  return DIAQ_OK;
}

// Modelled time of a plan in units of one pass over the state: an operation
// of at most four qubits costs its memory pass; a dense five-qubit group's
// 4096 FMAs per coset take longer than that pass (n = 28: 1.85 against
// 1.44 ms in complex128; in complex64, whose narrower groups run about
// 0.8 ms per pass, 1.45 ms on the vector kernels), less on the pipelined
// matrix cores, which take the groups whose qubits are all >= 4.
double plan_cost(const std::vector<BigOp>& ops, diaq_dtype_t dt, int n) {
  const double five = dt == DIAQ_C128 ? 1.3 : 1.8;
  double c = 0;
  // on the pipelined matrix cores (groups whose qubits are all >= 4):
  // complex64 one pass (n = 28: 0.87 ms, as a four-qubit group),
  // complex128 1.2 (1.74 ms)
  const double five_mfma = dt == DIAQ_C128 ? 1.2 : 1.0;
  for (const BigOp& op : ops) {
    if (op.raw || op.k != 5) c += 1.0;
    else c += mfma_group(op.q, op.k, n) ? five_mfma : five;
  }
  return c;
}

}  // namespace

diaq_status_t plan_big(const diaq_gate_t* gates, int64_t ngates, int n, int kmax, std::vector<BigOp>* ops,
                       diaq_dtype_t dt) {
  if (kmax < 1 || kmax > 5) return fail(DIAQ_ERR_INVALID_ARGUMENT, "max_fused_qubits must be 1..5");
  DIAQ_TRY(plan_big_greedy(gates, ngates, n, kmax, ops));
  // groups of up to five qubits: the greedy grouping with a narrower limit
  // can be cheaper (fewer five-qubit groups for few operations saved);
  // keep the plan of least modelled time (QFT-29: 24 operations with five
  // qubits against 25 with three, 97 against 81 ms)
  if (kmax == 5) {
    double best = plan_cost(*ops, dt, n);
    for (int k : {4, 3}) {
      std::vector<BigOp> alt;
      DIAQ_TRY(plan_big_greedy(gates, ngates, n, k, &alt));
      const double c = plan_cost(alt, dt, n);
      if (c < best) {
        best = c;
        ops->swap(alt);
      }
    }
  }
  return DIAQ_OK;
}

diaq_status_t run_big(diaq_ctx* ctx, const std::vector<BigOp>& ops, int n, diaq_dtype_t dt, void* state) {
  const int64_t N = int64_t(1) << n;
  // one table: every operation's matrix (2 D^2 doubles), then the factors
  std::vector<double> mats;
  std::vector<size_t> moff(ops.size()), loff(ops.size(), SIZE_MAX);
  OpTables tabs;
  const bool use_mfma = ctx->tuning.kron_split == 4 || ctx->tuning.kron_split == 5;
  const bool g3 = ctx->tuning.kron_split == 6;
  // pipelined matrix-core groups (all qubits >= 4): knob 7, and by default
  // complex64 groups of four and five qubits and complex128 groups of five
  // (n = 28, mean over positions: complex64 five qubits 1465 -> 869 us,
  // four 921 -> 891 us; complex128 five 1969 -> 1738 us, while its four-
  // qubit groups stay faster on the split kernel, 6.1 against 4.9 TB/s)
  auto use_mfmap = [&](const BigOp& op) {
    if (op.raw || !mfma_group(op.q, op.k, n)) return false;
    const int ks = ctx->tuning.kron_split;
    return ks == 7 || (ks == 0 && (dt == DIAQ_C64 || op.k == 5));
  };
  std::vector<size_t> loff3(ops.size(), SIZE_MAX), loffp(ops.size(), SIZE_MAX);
  for (size_t k = 0; k < ops.size(); k++) {
    moff[k] = mats.size();
    for (const Cd& z : ops[k].m) {
      mats.push_back(z.real());
      mats.push_back(z.imag());
    }
    if (g3 && !ops[k].raw && ops[k].k == 5) {
      // (Re, Im, Re + Im) per entry for the three-multiplication product
      loff3[k] = mats.size();
      for (const Cd& z : ops[k].m) {
        mats.push_back(z.real());
        mats.push_back(z.imag());
        mats.push_back(z.real() + z.imag());
      }
    }
    if (use_mfma && !ops[k].raw && mfma_group(ops[k].q, ops[k].k, n)) {
      // the real form in operand order, 16-byte aligned
      if (mats.size() & 1) mats.push_back(0.0);
      loff[k] = mats.size();
      const std::vector<double> lm = mfma_operands(ops[k].m, ops[k].k);
      mats.insert(mats.end(), lm.begin(), lm.end());
    }
    if (use_mfmap(ops[k])) {
      // the operands in the state's precision (complex64: fp32, two per
      // double slot), 16-byte aligned
      if (mats.size() & 1) mats.push_back(0.0);
      loffp[k] = mats.size();
      const std::vector<double> lm = mfmap_operands(ops[k].m, ops[k].k);
      if (dt == DIAQ_C128) {
        mats.insert(mats.end(), lm.begin(), lm.end());
      } else {
        std::vector<float> lf(lm.begin(), lm.end());
        const size_t at = mats.size();
        mats.resize(at + (lf.size() + 1) / 2, 0.0);
        std::memcpy(mats.data() + at, lf.data(), lf.size() * sizeof(float));
      }
    }
    // headers with the index bits of the operation's 2^k row offsets, for
    // kernels that decode each table once per coset
    int64_t off[32] = {0};
    const int nrows = ops[k].raw ? 0 : (1 << ops[k].k);
    for (int r = 0; r < nrows; r++)
      for (int j = 0; j < ops[k].k; j++)
        if ((r >> j) & 1) off[r] |= int64_t(1) << ops[k].q[j];
    tabs.add(ops[k].post, nrows ? off : nullptr, nrows);
  }
  const size_t mb = ((mats.size() * sizeof(double) + 255) / 256) * 256;
  const size_t bytes = mb + tabs.bytes.size() + 256;
  DIAQ_TRY(ensure(ctx, &ctx->aux, bytes));
  char* base = static_cast<char*>(ctx->aux.ptr);
  DIAQ_TRY(upload(ctx, base, mats.data(), mats.size() * sizeof(double)));
  DIAQ_TRY(upload(ctx, base + mb, tabs.bytes.data(), tabs.bytes.size()));
  const double* dm = reinterpret_cast<const double*>(base);
  const double bytes_op = 2.0 * double(elem_bytes(dt)) * double(N);
  for (size_t k = 0; k < ops.size(); k++) {
    const BigOp& op = ops[k];
    const int nt = tabs.count[k];
    const char* tk = nt ? base + mb + tabs.first[k] : nullptr;
    const size_t e0 = prof_mark(ctx);
    LdsArgs la;
    // complex128 state streams with non-temporal hints up to four qubits
    // (layered n = 28, groups of 4: 163 -> 155 ms); five-qubit groups
    // measured faster without
    const int ntp = (op.k <= 4 && dt == DIAQ_C128) ? 1 : 0;
    // dense 4-5 qubit groups: complex128 splits the rows over the waves of a
    // block by default (n = 28, mean over positions: four qubits with 4 rows
    // per wave 5.46 -> 6.00 TB/s, five qubits with 8 rows 4.54 -> 4.70);
    // complex64 keeps one lane per coset (its fp64 arithmetic, not memory,
    // is the limit: split 4.21 against 4.76 TB/s for four qubits) where the
    // pipelined fp32 matrix-core kernel does not apply (a qubit below 4)
    int split = ctx->tuning.kron_split;
    if (split == 0 || split == 7) split = dt == DIAQ_C128 ? (op.k == 4 ? 3 : 2) : 1;
    if (op.raw) {
      DIAQ_TRY(launch_kron_apply(ctx, ctx->stream, op.lg, n, dt, state, false, tk, nt));
    } else if (loffp[k] != SIZE_MAX) {
      // dense 4-5 qubit groups on the matrix cores, pipelined
      MfmaArgs ma;
      std::memset(&ma, 0, sizeof(ma));
      ma.ntiles = (N >> op.k) / 16;
      ma.nt = nt;
      ma.nt_io = ntp;
      for (int j = 0; j < op.k; j++) ma.sorted[j] = op.q[j];
      for (int r = 0; r < (1 << op.k); r++) {
        int64_t o = 0;
        for (int j = 0; j < op.k; j++)
          if ((r >> j) & 1) o |= int64_t(1) << op.q[j];
        ma.off[r] = o;
      }
      ma.lmat = dm + loffp[k];
      ma.tabs = tk;
      if (dt == DIAQ_C128) launch_mfmap<double>(ma, op.k, ctx->num_cus, ctx->stream, state);
      else launch_mfmap<float>(ma, op.k, ctx->num_cus, ctx->stream, state);
      DIAQ_HIP(hipGetLastError());
    } else if (loff[k] != SIZE_MAX) {
      // dense 4-5 qubit groups on the matrix cores
      MfmaArgs ma;
      std::memset(&ma, 0, sizeof(ma));
      ma.ntiles = (N >> op.k) / 16;
      ma.nt = nt;
      ma.nt_io = ntp;
      for (int j = 0; j < op.k; j++) ma.sorted[j] = op.q[j];
      for (int r = 0; r < (1 << op.k); r++) {
        int64_t o = 0;
        for (int j = 0; j < op.k; j++)
          if ((r >> j) & 1) o |= int64_t(1) << op.q[j];
        ma.off[r] = o;
      }
      ma.lmat = dm + loff[k];
      ma.tabs = tk;
      const bool hold = ctx->tuning.kron_split == 5;
      if (dt == DIAQ_C128) launch_mfma<double>(ma, op.k, hold, ctx->num_cus, ctx->stream, state);
      else launch_mfma<float>(ma, op.k, hold, ctx->num_cus, ctx->stream, state);
      DIAQ_HIP(hipGetLastError());
    } else if (op.k >= 4 && split >= 2 && split != 4 && split != 5 && make_lds_args(op.q, op.k, n, &la)) {
      // dense 4-5 qubit groups, rows split over the waves of a block
      const bool three = loff3[k] != SIZE_MAX;
      la.mat = dm + (three ? loff3[k] : moff[k]);
      la.tabs = tk;
      la.nt = nt;
      la.nt_io = ntp;
      la.order = group_order(ctx->tuning);
      const int rows = split == 3 ? 4 : 8;
      if (dt == DIAQ_C128) launch_split<double>(la, op.k, rows, three, n, ctx->stream, state);
      else launch_split<float>(la, op.k, rows, three, n, ctx->stream, state);
      DIAQ_HIP(hipGetLastError());
    } else if (staged(op.q, op.k, stage_low(ctx->tuning, dt)) && make_lds_args(op.q, op.k, n, &la)) {
      la.mat = dm + moff[k];
      la.tabs = tk;
      la.nt = nt;
      la.nt_io = ntp;
      la.order = group_order(ctx->tuning);
      if (dt == DIAQ_C128) launch_lds<double>(la, op.k, n, ctx->stream, state);
      else launch_lds<float>(la, op.k, n, ctx->stream, state);
      DIAQ_HIP(hipGetLastError());
    } else if (op.k <= 3) {
      // small groups: the three-qubit kernels, controls already in the matrix
      LocalGate lg;
      std::memset(&lg, 0, sizeof(lg));
      lg.k = op.k;
      const int D = 1 << op.k;
      for (int j = 0; j < op.k; j++) {
        lg.targets[j] = op.q[j];
        lg.tmask |= uint64_t(1) << op.q[j];
      }
      for (int r = 0; r < D; r++)
        for (int c = 0; c < D; c++) {
          const Cd z = op.m[size_t(r) * D + c];
          lg.m[r][c][0] = z.real();
          lg.m[r][c][1] = z.imag();
          lg.structural[r][c] = z != Cd(0, 0);
        }
      DIAQ_TRY(launch_kron_apply(ctx, ctx->stream, lg, n, dt, state, false, tk, nt));
    } else {
      BigArgs a;
      std::memset(&a, 0, sizeof(a));
      a.ncos = N >> op.k;
      a.nt = nt;
      a.nt_io = ntp;
      for (int j = 0; j < op.k; j++) a.sorted[j] = op.q[j];
      for (int r = 0; r < (1 << op.k); r++) {
        int64_t o = 0;
        for (int j = 0; j < op.k; j++)
          if ((r >> j) & 1) o |= int64_t(1) << op.q[j];
        a.off[r] = o;
      }
      a.mat = dm + moff[k];
      a.tabs = tk;
      const dim3 grid(unsigned((a.ncos + kBigBlock - 1) / kBigBlock)), block(kBigBlock);
      if (dt == DIAQ_C128) {
        if (op.k == 4) hipLaunchKernelGGL((kron_big_kernel<double, 4>), grid, block, 0, ctx->stream, a,
                                          static_cast<double2*>(state));
        else hipLaunchKernelGGL((kron_big_kernel<double, 5>), grid, block, 0, ctx->stream, a,
                                static_cast<double2*>(state));
      } else {
        if (op.k == 4) hipLaunchKernelGGL((kron_big_kernel<float, 4>), grid, block, 0, ctx->stream, a,
                                          static_cast<float2*>(state));
        else hipLaunchKernelGGL((kron_big_kernel<float, 5>), grid, block, 0, ctx->stream, a,
                                static_cast<float2*>(state));
      }
      DIAQ_HIP(hipGetLastError());
    }
    prof_interval(ctx, e0, prof_mark(ctx), 1, bytes_op);
  }
  return DIAQ_OK;
}

}  // namespace diaq

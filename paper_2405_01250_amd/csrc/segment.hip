// segment.hip -- the adjoint reverse sweep with many gates per pass.
//
// The reverse sweep needs, for every differentiable gate g (in reverse
// order), the dot <lambda|G_g|psi> at the point right after g, and then
// psi, lambda <- U_g^dagger (the transpose-and-conjugate of Sec. IV).  Done
// gate by gate that is four vector streams per gate.  Here the sweep is cut
// into segments of consecutive gates whose non-diagonal targets fit in three
// qubits S; diagonal gates (and the controls of any gate) may sit on any
// qubit.  One lane owns a coset of S (8 amplitudes of psi and of lambda, the
// cosets of Alg. 3) and replays the segment's gates on it in exact reverse
// order, taking each gate's dot before undoing it.  Every amplitude of psi
// and lambda is then read and written once per segment instead of once per
// gate, and nothing is reordered, so the result is the gate-by-gate sweep
// up to rounding.
//
// Dots: each wave reduces its lanes' contributions with shuffles and parks
// the sum in LDS; the workgroup writes one partial per dot, and a second
// kernel sums the partials over workgroups in a fixed order.
//
// A forward plan is the same cut taken in circuit order with U instead of
// U^dagger and psi alone: the batched path uses it so that one table of
// per-gate matrices (refreshed on the device from new angles) serves both
// passes.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace diaq {

namespace {

constexpr int kSegBlock = 256;
constexpr int kSegWaves = kSegBlock / 64;
static_assert(sizeof(SegGate) % sizeof(uint64_t) == 0, "SegGate is copied in 8-byte words");

enum SegKind : int32_t { kOne = 0, kTwo = 1, kThree = 2, kDiag = 3, kRun = 4, kRunMember = 5 };

struct SegArgs {
  int64_t ncos;        // N / 8
  int32_t sorted[3];   // S ascending
  int32_t ngates;
  int32_t ndots;
  int32_t tables;      // 1: diagonal gates, whose tables are staged in LDS
  int64_t off[8];      // global offset of local index r
  const SegGate* gates;
  const double* pool;
  int64_t pool_lo;     // the segment's matrices: pool[pool_lo, pool_lo + pool_n)
  int64_t pool_n;
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

struct Coset {
  double pr[8], pi[8], lr[8], li[8];
};

// The segment's gate list and matrices are read where the host (or the
// batch's angle refresh, an earlier kernel) wrote them, through the
// constant address space: every lane reads the same gate and the same
// matrix entries, so these become scalar loads whose values feed the FMAs
// from SGPRs (staging them in LDS made each entry a 64-lane LDS read, as
// much LDS traffic per coset as the state moves to HBM).  The per-row
// entries of diagonal tables differ by lane and stay vector loads.
typedef __attribute__((address_space(4))) const double CD;
typedef __attribute__((address_space(4))) const SegGate CG;

// Gate i of the list, field by field through the constant address space.
__device__ __forceinline__ SegGate seg_gate(const SegGate* gates, int i) {
  CG* p = (CG*)(gates) + i;
  SegGate g;
  g.kind = p->kind;
  g.b0 = p->b0;
  g.b1 = p->b1;
  g.dot = p->dot;
  g.dk = p->dk;
  g.q[0] = p->q[0];
  g.q[1] = p->q[1];
  g.q[2] = p->q[2];
  g.cmask = p->cmask;
  g.moff = p->moff;
  return g;
}

// y = M x on the local indices idx[0..D) of the coset, for psi and lambda,
// after the dot conj(lambda) (G psi) when G != nullptr.
template <int D, bool LAM, typename P>
__device__ __forceinline__ void local_apply(Coset& s, const int (&idx)[D], P m, P g, double& dre, double& dim) {
  if (LAM && g) {
#pragma unroll
    for (int r = 0; r < D; r++) {
      double gr = 0, gi = 0;
#pragma unroll
      for (int c = 0; c < D; c++) {
        const double a = g[(r * D + c) * 2], b = g[(r * D + c) * 2 + 1];
        gr += a * s.pr[idx[c]] - b * s.pi[idx[c]];
        gi += a * s.pi[idx[c]] + b * s.pr[idx[c]];
      }
      dre += s.lr[idx[r]] * gr + s.li[idx[r]] * gi;
      dim += s.lr[idx[r]] * gi - s.li[idx[r]] * gr;
    }
  }
  double yr[D], yi[D], zr[D], zi[D];
#pragma unroll
  for (int r = 0; r < D; r++) {
    double ar = 0, ai = 0, br = 0, bi = 0;
#pragma unroll
    for (int c = 0; c < D; c++) {
      const double a = m[(r * D + c) * 2], b = m[(r * D + c) * 2 + 1];
      ar += a * s.pr[idx[c]] - b * s.pi[idx[c]];
      ai += a * s.pi[idx[c]] + b * s.pr[idx[c]];
      if (LAM) {
        br += a * s.lr[idx[c]] - b * s.li[idx[c]];
        bi += a * s.li[idx[c]] + b * s.lr[idx[c]];
      }
    }
    yr[r] = ar;
    yi[r] = ai;
    zr[r] = br;
    zi[r] = bi;
  }
#pragma unroll
  for (int r = 0; r < D; r++) {
    s.pr[idx[r]] = yr[r];
    s.pi[idx[r]] = yi[r];
    if (LAM) {
      s.lr[idx[r]] = zr[r];
      s.li[idx[r]] = zi[r];
    }
  }
}

// One-target gate on local bit B: four pairs (r, r | 1 << B).
template <int B, bool LAM>
__device__ __forceinline__ void apply_one(Coset& s, const SegArgs& a, const double* pool, const SegGate& sg, int64_t base,
                                          double& dre, double& dim) {
  CD* m = (CD*)(pool + sg.moff);
  CD* g = sg.dot >= 0 ? m + 8 : nullptr;
#pragma unroll
  for (int p = 0; p < 4; p++) {
    const int r0 = ((p >> B) << (B + 1)) | (p & ((1 << B) - 1));
    const int idx[2] = {r0, r0 | (1 << B)};
    if (sg.cmask && ((uint64_t(base + a.off[r0]) & sg.cmask) != sg.cmask)) continue;
    local_apply<2, LAM>(s, idx, m, g, dre, dim);
  }
}

// Two-target gate: target 0 on local bit B0, target 1 on B1; two quads.
template <int B0, int B1, bool LAM>
__device__ __forceinline__ void apply_two(Coset& s, const SegArgs& a, const double* pool, const SegGate& sg, int64_t base,
                                          double& dre, double& dim) {
  constexpr int FREE = 7 & ~((1 << B0) | (1 << B1));
  CD* m = (CD*)(pool + sg.moff);
  CD* g = sg.dot >= 0 ? m + 32 : nullptr;
#pragma unroll
  for (int p = 0; p < 2; p++) {
    const int r0 = p ? FREE : 0;
    const int idx[4] = {r0, r0 | (1 << B0), r0 | (1 << B1), r0 | (1 << B0) | (1 << B1)};
    if (sg.cmask && ((uint64_t(base + a.off[r0]) & sg.cmask) != sg.cmask)) continue;
    local_apply<4, LAM>(s, idx, m, g, dre, dim);
  }
}

template <bool LAM>
__device__ __forceinline__ void apply_three(Coset& s, const double* pool, const SegGate& sg, int64_t base, double& dre,
                                            double& dim) {
  if (sg.cmask && ((uint64_t(base) & sg.cmask) != sg.cmask)) return;
  CD* m = (CD*)(pool + sg.moff);
  CD* g = sg.dot >= 0 ? m + 128 : nullptr;
  const int idx[8] = {0, 1, 2, 3, 4, 5, 6, 7};
  local_apply<8, LAM>(s, idx, m, g, dre, dim);
}

// Diagonal gate on any qubits: each amplitude reads its entry of the
// gate's (at most 8-entry) table.
template <bool LAM>
__device__ __forceinline__ void apply_diag(Coset& s, const SegArgs& a, const double* tabs, const SegGate& sg,
                                           int64_t base, double& dre, double& dim) {
  const double* v = tabs + sg.moff;
  const double* g = v + 2 * (1 << sg.dk);
#pragma unroll
  for (int r = 0; r < 8; r++) {
    const uint64_t i = uint64_t(base + a.off[r]);
    if ((i & sg.cmask) != sg.cmask) continue;
    int t = 0;
#pragma unroll
    for (int j = 0; j < 3; j++)
      if (j < sg.dk) t |= int((i >> sg.q[j]) & 1) << j;
    if (LAM && sg.dot >= 0) {
      const double gr = g[2 * t] * s.pr[r] - g[2 * t + 1] * s.pi[r];
      const double gi = g[2 * t] * s.pi[r] + g[2 * t + 1] * s.pr[r];
      dre += s.lr[r] * gr + s.li[r] * gi;
      dim += s.lr[r] * gi - s.li[r] * gr;
    }
    const double vr = v[2 * t], vi = v[2 * t + 1];
    double x = vr * s.pr[r] - vi * s.pi[r];
    s.pi[r] = vr * s.pi[r] + vi * s.pr[r];
    s.pr[r] = x;
    if (LAM) {
      x = vr * s.lr[r] - vi * s.li[r];
      s.li[r] = vr * s.li[r] + vi * s.lr[r];
      s.lr[r] = x;
    }
  }
}

// Wave sum of one dot, parked in LDS for the workgroup's partial.
__device__ __forceinline__ void flush_dot(double2 (*acc)[kSegBlock / 64], int j, double dre, double dim) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    dre += __shfl_xor(dre, o, 64);
    dim += __shfl_xor(dim, o, 64);
  }
  if ((threadIdx.x & 63) == 0) acc[j][threadIdx.x >> 6] = double2{dre, dim};
}

// A run of m diagonal gates (the m entries after the header).  They commute,
// so every dot may be taken at the start of the run, where it is
// sum_i G(i) conj(lambda_i) psi_i (the generators are real and diagonal);
// the phases multiply into one factor per amplitude, applied once.
// Consecutive members that share a dot slot (same parameter and scale) add
// into one dot.
template <bool LAM>
__device__ __forceinline__ void apply_run(Coset& s, const SegArgs& a, const SegGate* gates, const double* tabs, int gi, int m,
                                          int64_t base, double2 (*acc)[kSegBlock / 64]) {
  double fr[8], fi[8];
#pragma unroll
  for (int r = 0; r < 8; r++) {
    fr[r] = 1.0;
    fi[r] = 0.0;
  }
  int cur = -1;
  double dre = 0, dim = 0;
  for (int k = 1; k <= m; k++) {
    const SegGate mg = seg_gate(gates, gi + k);
    if (LAM && mg.dot >= 0 && mg.dot != cur) {
      if (cur >= 0) flush_dot(acc, cur, dre, dim);
      cur = mg.dot;
      dre = dim = 0;
    }
    const double* vt = tabs + mg.moff;
    const double* gt = vt + 2 * (1 << mg.dk);
#pragma unroll
    for (int r = 0; r < 8; r++) {
      const uint64_t i = uint64_t(base + a.off[r]);
      if ((i & mg.cmask) != mg.cmask) continue;
      int t = 0;
#pragma unroll
      for (int j = 0; j < 3; j++)
        if (j < mg.dk) t |= int((i >> mg.q[j]) & 1) << j;
      const double vr = vt[2 * t], vi = vt[2 * t + 1];
      const double x = fr[r] * vr - fi[r] * vi;
      fi[r] = fr[r] * vi + fi[r] * vr;
      fr[r] = x;
      if (LAM && mg.dot >= 0) {
        // conj(lambda) psi, unchanged by the run's phases (recomputed here
        // rather than held in registers)
        const double g = gt[t];
        dre += g * (s.lr[r] * s.pr[r] + s.li[r] * s.pi[r]);
        dim += g * (s.lr[r] * s.pi[r] - s.li[r] * s.pr[r]);
      }
    }
  }
  if (LAM && cur >= 0) flush_dot(acc, cur, dre, dim);
#pragma unroll
  for (int r = 0; r < 8; r++) {
    double x = fr[r] * s.pr[r] - fi[r] * s.pi[r];
    s.pi[r] = fr[r] * s.pi[r] + fi[r] * s.pr[r];
    s.pr[r] = x;
    if (LAM) {
      x = fr[r] * s.lr[r] - fi[r] * s.li[r];
      s.li[r] = fr[r] * s.li[r] + fi[r] * s.lr[r];
      s.lr[r] = x;
    }
  }
}

// One workgroup's share of a segment pass: workgroup `block` of the grid
// over a's cosets.
template <typename R, bool LAM, bool T3>
__device__ __forceinline__ void segment_body(const SegArgs& ga, typename Vec<R>::V* psi_in,
                                             typename Vec<R>::V* lam_in, double2* partial_in, int64_t block) {
  using NV = typename Nat<R>::T;
  using ND = typename Nat<double>::T;
  auto* __restrict__ psi = gptr(reinterpret_cast<NV*>(psi_in));
  auto* __restrict__ lam = gptr(reinterpret_cast<NV*>(lam_in));
  auto* __restrict__ partial = gptr(reinterpret_cast<ND*>(partial_in));
  __shared__ double2 acc[kSegMaxDots][kSegWaves];
  // the tables of diagonal gates, staged in LDS (their entries differ by
  // lane); dense matrices and the gate list are read through scalar loads
  __shared__ double lpool[kSegLdsPool];
  const SegArgs& a = ga;
  const SegGate* gates = ga.gates;
  const double* pool = ga.pool;
  const double* tabs = lpool - ga.pool_lo;
  const int64_t c = block * kSegBlock + threadIdx.x;
  const bool live = c < a.ncos;
  int64_t base = 0;
  if (live) {
    base = c;
#pragma unroll
    for (int j = 0; j < 3; j++) {
      const int p = a.sorted[j];
      base = (base & ((int64_t(1) << p) - 1)) | ((base >> p) << (p + 1));
    }
  }
  // the state loads go out first; the staging below overlaps their latency
  Coset s;
#pragma unroll
  for (int r = 0; r < 8; r++) {
    NV x = live ? psi[base + a.off[r]] : NV{R(0), R(0)};
    NV y = (LAM && live) ? lam[base + a.off[r]] : NV{R(0), R(0)};
    s.pr[r] = double(x.x);
    s.pi[r] = double(x.y);
    s.lr[r] = double(y.x);
    s.li[r] = double(y.y);
  }
  if (ga.tables) {
    const auto* src = gptr(ga.pool);
    for (int t = threadIdx.x; t < int(ga.pool_n); t += kSegBlock) lpool[t] = src[ga.pool_lo + t];
    __syncthreads();
  }
  for (int gi = 0; gi < a.ngates; gi++) {
    const SegGate sg = seg_gate(gates, gi);
    if (sg.kind == kRun) {
      apply_run<LAM>(s, a, gates, tabs, gi, sg.b0, base, acc);
      gi += sg.b0;
      continue;
    }
    double dre = 0, dim = 0;
    if (live) {
      switch (sg.kind) {
        case kOne:
          if (sg.b0 == 0) apply_one<0, LAM>(s, a, pool, sg, base, dre, dim);
          else if (sg.b0 == 1) apply_one<1, LAM>(s, a, pool, sg, base, dre, dim);
          else apply_one<2, LAM>(s, a, pool, sg, base, dre, dim);
          break;
        case kTwo: {
          const int code = sg.b0 * 3 + sg.b1;
          switch (code) {
            case 1: apply_two<0, 1, LAM>(s, a, pool, sg, base, dre, dim); break;
            case 2: apply_two<0, 2, LAM>(s, a, pool, sg, base, dre, dim); break;
            case 3: apply_two<1, 0, LAM>(s, a, pool, sg, base, dre, dim); break;
            case 5: apply_two<1, 2, LAM>(s, a, pool, sg, base, dre, dim); break;
            case 6: apply_two<2, 0, LAM>(s, a, pool, sg, base, dre, dim); break;
            default: apply_two<2, 1, LAM>(s, a, pool, sg, base, dre, dim); break;
          }
          break;
        }
        case kThree:
          if constexpr (T3) apply_three<LAM>(s, pool, sg, base, dre, dim);
          break;
        default:
          apply_diag<LAM>(s, a, tabs, sg, base, dre, dim);
          break;
      }
    }
    if (LAM && sg.dot >= 0) flush_dot(acc, sg.dot, dre, dim);
  }
  if (live) {
#pragma unroll
    for (int r = 0; r < 8; r++) {
      psi[base + a.off[r]] = NV{R(s.pr[r]), R(s.pi[r])};
      if (LAM) lam[base + a.off[r]] = NV{R(s.lr[r]), R(s.li[r])};
    }
  }
  if (!LAM) return;
  __syncthreads();
  for (int j = threadIdx.x; j < a.ndots; j += kSegBlock) {
    double2 t = acc[j][0];
    for (int w = 1; w < kSegWaves; w++) {
      t.x += acc[j][w].x;
      t.y += acc[j][w].y;
    }
    partial[block * a.ndots + j] = ND{t.x, t.y};
  }
}

template <typename R, bool LAM, bool T3>
__global__ __launch_bounds__(kSegBlock, LAM ? 3 : 1) void segment_kernel(SegArgs a, typename Vec<R>::V* __restrict__ psi,
                                                            typename Vec<R>::V* __restrict__ lam,
                                                            double2* __restrict__ partial) {
  segment_body<R, LAM, T3>(a, psi, lam, partial, blockIdx.x);
}

// Grouped launch: segment passes over many independent states in one grid;
// each state's workgroups follow the previous state's.
struct GroupSeg {
  SegArgs a;
  void* psi;
  void* lam;
  double2* partial;
  int64_t block0;
};

template <typename R, bool LAM, bool T3>
__global__ __launch_bounds__(kSegBlock, LAM ? 3 : 1) void grouped_segment_kernel(const GroupSeg* __restrict__ list, int count) {
  int lo = 0, hi = count - 1;  // last item with block0 <= blockIdx.x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (list[mid].block0 <= int64_t(blockIdx.x)) lo = mid;
    else hi = mid - 1;
  }
  const GroupSeg& g = list[lo];
  segment_body<R, LAM, T3>(g.a, static_cast<typename Vec<R>::V*>(g.psi), static_cast<typename Vec<R>::V*>(g.lam),
                           g.partial, int64_t(blockIdx.x) - g.block0);
}

// Dot j of a segment: the partials of all workgroups summed in a fixed
// order, written to out[2 * slot[j]].
__global__ __launch_bounds__(256) void segment_reduce_kernel(const double2* __restrict__ partial, int64_t blocks,
                                                             int32_t ndots, const int64_t* __restrict__ slot,
                                                             double* __restrict__ out) {
  const int j = blockIdx.x;
  double re = 0, im = 0;
  for (int64_t b = threadIdx.x; b < blocks; b += 256) {
    re += partial[b * ndots + j].x;
    im += partial[b * ndots + j].y;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    re += __shfl_xor(re, o, 64);
    im += __shfl_xor(im, o, 64);
  }
  __shared__ double2 ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = double2{re, im};
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 t = ws[0];
    for (int w = 1; w < 4; w++) {
      t.x += ws[w].x;
      t.y += ws[w].y;
    }
    out[2 * slot[j]] = t.x;
    out[2 * slot[j] + 1] = t.y;
  }
}

template <typename R, bool T3>
void launch_segment(bool forward, int64_t blocks, hipStream_t stream, const SegArgs& a, void* psi, void* lam,
                    double2* partial) {
  using V = typename Vec<R>::V;
  if (forward)
    hipLaunchKernelGGL((segment_kernel<R, false, T3>), dim3(unsigned(blocks)), dim3(kSegBlock), 0, stream, a,
                       static_cast<V*>(psi), nullptr, nullptr);
  else
    hipLaunchKernelGGL((segment_kernel<R, true, T3>), dim3(unsigned(blocks)), dim3(kSegBlock), 0, stream, a,
                       static_cast<V*>(psi), static_cast<V*>(lam), partial);
}

// Grouped dot sums: workgroup b handles dot (b - red0) of its item.
struct GroupRed {
  const double2* partial;
  int64_t blocks;
  int32_t ndots;
  int32_t pad;
  const int64_t* slot;
  int64_t red0;
};

__global__ __launch_bounds__(256) void grouped_reduce_kernel(const GroupRed* __restrict__ list, int count,
                                                             double* __restrict__ out) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (list[mid].red0 <= int64_t(blockIdx.x)) lo = mid;
    else hi = mid - 1;
  }
  const GroupRed& g = list[lo];
  const int j = int(int64_t(blockIdx.x) - g.red0);
  const auto* part = gptr(reinterpret_cast<const typename Nat<double>::T*>(g.partial));
  double re = 0, im = 0;
  for (int64_t b = threadIdx.x; b < g.blocks; b += 256) {
    const auto v = part[b * g.ndots + j];
    re += v.x;
    im += v.y;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    re += __shfl_xor(re, o, 64);
    im += __shfl_xor(im, o, 64);
  }
  __shared__ double2 ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = double2{re, im};
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 t = ws[0];
    for (int w = 1; w < 4; w++) {
      t.x += ws[w].x;
      t.y += ws[w].y;
    }
    const int64_t sl = gptr(g.slot)[j];
    out[2 * sl] = t.x;
    out[2 * sl + 1] = t.y;
  }
}

SegArgs make_seg_args(const SegmentPlan& P, const Segment& seg, int n, const SegGate* dg, const double* dp) {
  SegArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ncos = (int64_t(1) << n) >> 3;
  for (int j = 0; j < 3; j++) a.sorted[j] = seg.S[j];
  for (int r = 0; r < 8; r++) {
    int64_t o = 0;
    for (int j = 0; j < 3; j++)
      if ((r >> j) & 1) o |= int64_t(1) << seg.S[j];
    a.off[r] = o;
  }
  a.ngates = int32_t(seg.ngates);
  a.ndots = seg.ndots;
  a.gates = dg + seg.first;
  a.pool = dp;
  a.pool_lo = seg.pool_lo;
  a.pool_n = seg.pool_n;
  for (int64_t g = 0; g < seg.ngates; g++) {
    const int32_t k = P.gates[size_t(seg.first + g)].kind;
    if (k == kDiag || k == kRun || k == kRunMember) a.tables = 1;
  }
  return a;
}

bool is_diag(const LocalGate& lg) {
  const int d = 1 << lg.k;
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++)
      if (r != c && lg.structural[r][c]) return false;
  return true;
}

// Padding qubits for a segment whose non-diagonal targets use fewer than
// three: middle qubits first (measured the best-coalesced cosets), then
// the rest.
void pad_set(std::vector<int>& S, int n) {
  std::vector<int> order;
  for (int q = std::min(10, n - 1); q < n; q++) order.push_back(q);
  for (int q = std::min(10, n - 1) - 1; q >= 0; q--) order.push_back(q);
  for (int q : order) {
    if (int(S.size()) == 3) break;
    if (std::find(S.begin(), S.end(), q) == S.end()) S.push_back(q);
  }
  std::sort(S.begin(), S.end());
}

// A diagonal gate that can join a run: its entries are pure phases and,
// when its dot is wanted, its generator is real.
bool run_member(const LocalGate& L, const LocalGate& gen, bool dot) {
  if (!is_diag(L)) return false;
  for (int r = 0; r < (1 << L.k); r++) {
    if (std::fabs(std::hypot(L.m[r][r][0], L.m[r][r][1]) - 1.0) > 1e-13) return false;
    if (dot && gen.m[r][r][1] != 0.0) return false;
  }
  return true;
}

int local_bit(const std::vector<int>& S, int q) {
  return int(std::find(S.begin(), S.end(), q) - S.begin());
}

}  // namespace

diaq_status_t plan_segments(const std::vector<LocalGate>& lg, const std::vector<LocalGate>& gens,
                            const std::vector<int64_t>& dkey, int n, SegmentPlan* out, bool forward) {
  if (n < 3) return fail(DIAQ_ERR_UNSUPPORTED, "segment sweep needs n >= 3");
  SegmentPlan& P = *out;
  P = SegmentPlan();
  P.forward = forward;
  const int64_t G = int64_t(lg.size());
  // the sweep visits gates from `g` towards `end` in steps of `dir`
  const int64_t dir = forward ? 1 : -1, end = forward ? G : -1;
  int64_t g = forward ? 0 : G - 1;
  while (g != end) {
    // grow the segment from gate g
    std::vector<int> S;
    std::vector<int64_t> members;
    int ndots = 0;
    int64_t pool_need = 0;
    for (; g != end; g += dir) {
      const LocalGate& L = lg[size_t(g)];
      std::vector<int> T;
      if (!is_diag(L))
        for (int j = 0; j < L.k; j++) T.push_back(L.targets[j]);
      std::vector<int> U = S;
      for (int q : T)
        if (std::find(U.begin(), U.end(), q) == U.end()) U.push_back(q);
      const bool want_dot = !forward && dkey[size_t(g)] >= 0;
      // LDS budget: entries (a run header at most every second member) and
      // matrix doubles (diagonal gates counted at their complex size)
      const int d = 1 << L.k;
      const int64_t need = (is_diag(L) ? 2 * d : 2 * d * d) * (want_dot ? 2 : 1);
      const int64_t entries = int64_t(members.size()) + 1;
      if (U.size() > 3 || entries + entries / 2 + 1 > kSegLdsGates || pool_need + need > kSegLdsPool ||
          (want_dot && ndots >= kSegMaxDots))
        break;
      S = U;
      members.push_back(g);
      pool_need += need;
      if (want_dot) ndots++;
    }
    pad_set(S, n);
    Segment seg;
    for (int j = 0; j < 3; j++) seg.S[j] = S[size_t(j)];
    seg.first = int64_t(P.gates.size());
    seg.pool_lo = int64_t(P.pool.size());
    seg.ndots = 0;
    seg.dot_slot0 = int64_t(P.dot_gate.size());
    auto push = [&](double re, double im) {
      P.pool.push_back(re);
      P.pool.push_back(im);
    };
    for (size_t mi = 0; mi < members.size();) {
      // a run of >= 2 consecutive diagonal phase gates becomes one kRun
      size_t mj = mi;
      while (mj < members.size() && run_member(lg[size_t(members[mj])], gens[size_t(members[mj])],
                                               !forward && dkey[size_t(members[mj])] >= 0))
        mj++;
      if (mj - mi >= 2) {
        SegGate hd;
        std::memset(&hd, 0, sizeof(hd));
        hd.kind = kRun;
        hd.b0 = int32_t(mj - mi);
        hd.dot = -1;
        P.gates.push_back(hd);
        P.gate_of.push_back(members[mi]);
        int64_t last_key = -1;
        int last_dot = -1;
        for (size_t x = mi; x < mj; x++) {
          const int64_t m = members[x];
          const LocalGate& L = lg[size_t(m)];
          SegGate sg;
          std::memset(&sg, 0, sizeof(sg));
          sg.kind = kRunMember;
          sg.cmask = L.cmask;
          sg.dk = L.k;
          for (int j = 0; j < L.k; j++) sg.q[j] = L.targets[j];
          sg.dot = -1;
          if (!forward && dkey[size_t(m)] >= 0) {
            if (dkey[size_t(m)] == last_key) {
              sg.dot = last_dot;
            } else {
              sg.dot = last_dot = seg.ndots++;
              last_key = dkey[size_t(m)];
              P.dot_gate.push_back(m);
            }
          }
          sg.moff = int64_t(P.pool.size());
          const int d = 1 << L.k;
          for (int r = 0; r < d; r++) push(L.m[r][r][0], forward ? L.m[r][r][1] : -L.m[r][r][1]);
          if (sg.dot >= 0)
            for (int r = 0; r < d; r++) P.pool.push_back(gens[size_t(m)].m[r][r][0]);
          P.gates.push_back(sg);
          P.gate_of.push_back(m);
        }
        mi = mj;
        continue;
      }
      const int64_t m = members[mi++];
      const LocalGate& L = lg[size_t(m)];
      SegGate sg;
      std::memset(&sg, 0, sizeof(sg));
      sg.cmask = L.cmask;
      sg.dot = (!forward && dkey[size_t(m)] >= 0) ? seg.ndots++ : -1;
      if (sg.dot >= 0) P.dot_gate.push_back(m);
      P.gate_of.push_back(m);
      sg.moff = int64_t(P.pool.size());
      const int d = 1 << L.k;
      if (is_diag(L)) {
        sg.kind = kDiag;
        sg.dk = L.k;
        for (int j = 0; j < L.k; j++) sg.q[j] = L.targets[j];
        for (int r = 0; r < d; r++) push(L.m[r][r][0], forward ? L.m[r][r][1] : -L.m[r][r][1]);
        if (sg.dot >= 0)
          for (int r = 0; r < d; r++) push(gens[size_t(m)].m[r][r][0], gens[size_t(m)].m[r][r][1]);
      } else {
        // local order: kOne / kTwo keep the gate's own order (b0, b1 say where
        // its targets sit in S); kThree is permuted into S's order
        int perm[8];
        for (int r = 0; r < d; r++) perm[r] = r;
        if (L.k == 1) {
          sg.kind = kOne;
          sg.b0 = local_bit(S, L.targets[0]);
        } else if (L.k == 2) {
          sg.kind = kTwo;
          sg.b0 = local_bit(S, L.targets[0]);
          sg.b1 = local_bit(S, L.targets[1]);
        } else {
          sg.kind = kThree;
          seg.three = true;
          // S-local index rs -> gate-local index
          for (int rs = 0; rs < 8; rs++) {
            int rg = 0;
            for (int j = 0; j < 3; j++)
              if ((rs >> j) & 1) rg |= 1 << (std::find(L.targets, L.targets + 3, S[size_t(j)]) - L.targets);
            perm[rs] = rg;
          }
        }
        for (int r = 0; r < d; r++)
          for (int c = 0; c < d; c++) {
            const int pr = perm[r], pc = perm[c];
            if (forward) push(L.m[pr][pc][0], L.m[pr][pc][1]);
            else push(L.m[pc][pr][0], -L.m[pc][pr][1]);  // U^dagger[r][c] = conj(U[c][r])
          }
        if (sg.dot >= 0)
          for (int r = 0; r < d; r++)
            for (int c = 0; c < d; c++) push(gens[size_t(m)].m[perm[r]][perm[c]][0],
                                              gens[size_t(m)].m[perm[r]][perm[c]][1]);
      }
      P.gates.push_back(sg);
    }
    seg.ngates = int64_t(P.gates.size()) - seg.first;
    seg.pool_n = int64_t(P.pool.size()) - seg.pool_lo;
    P.segs.push_back(seg);
  }
  return DIAQ_OK;
}

diaq_status_t run_segments(diaq_ctx* ctx, hipStream_t stream, const SegmentPlan& P, int n, diaq_dtype_t dt,
                           void* psi, void* lam, void* table_mem, double2* partial, double* dots) {
  // table_mem: device copy of [gates | pool | dot slots | reduce records],
  // laid out by segment_table_bytes; each segment's partial sums have their
  // own rows of `partial` (segment_partial_entries), so all dot sums run in
  // one launch after the sweep
  char* t = static_cast<char*>(table_mem);
  const size_t gb = ((P.gates.size() * sizeof(SegGate) + 255) / 256) * 256;
  const SegGate* dg = reinterpret_cast<const SegGate*>(t);
  const double* dp = reinterpret_cast<const double*>(t + gb);
  const int64_t blocks = segment_blocks(n);
  int64_t row = 0, ndots = 0, nred = 0;
  for (const Segment& seg : P.segs) {
    const SegArgs a = make_seg_args(P, seg, n, dg, dp);
    double2* part = partial + row;
    if (dt == DIAQ_C128) {
      if (seg.three) launch_segment<double, true>(P.forward, blocks, stream, a, psi, lam, part);
      else launch_segment<double, false>(P.forward, blocks, stream, a, psi, lam, part);
    } else {
      if (seg.three) launch_segment<float, true>(P.forward, blocks, stream, a, psi, lam, part);
      else launch_segment<float, false>(P.forward, blocks, stream, a, psi, lam, part);
    }
    DIAQ_HIP(hipGetLastError());
    row += blocks * seg.ndots;
    ndots += seg.ndots;
    nred += seg.ndots ? 1 : 0;
  }
  if (ndots) {
    const GroupRed* reds = reinterpret_cast<const GroupRed*>(t + segment_reds_offset(P));
    hipLaunchKernelGGL(grouped_reduce_kernel, dim3(unsigned(ndots)), dim3(256), 0, stream, reds, int(nred), dots);
    DIAQ_HIP(hipGetLastError());
  }
  return DIAQ_OK;
}

int64_t segment_partial_entries(const SegmentPlan& P, int n) {
  int64_t e = 0;
  for (const Segment& seg : P.segs) e += segment_blocks(n) * seg.ndots;
  return std::max<int64_t>(e, 1);
}

size_t segment_reds_offset(const SegmentPlan& P) {
  const size_t gb = ((P.gates.size() * sizeof(SegGate) + 255) / 256) * 256;
  const size_t pb = ((P.pool.size() * sizeof(double) + 255) / 256) * 256;
  return gb + pb + ((P.dot_gate.size() * sizeof(int64_t) + 255) / 256) * 256;
}

void segment_table_reds(const SegmentPlan& P, int n, const void* table_dev, const double2* partial,
                        std::vector<char>& host) {
  const char* t = static_cast<const char*>(table_dev);
  const size_t gb = ((P.gates.size() * sizeof(SegGate) + 255) / 256) * 256;
  const size_t pb = ((P.pool.size() * sizeof(double) + 255) / 256) * 256;
  const size_t ro = segment_reds_offset(P);
  int64_t row = 0, red0 = 0;
  size_t k = 0;
  for (const Segment& seg : P.segs) {
    if (seg.ndots) {
      GroupRed r;
      std::memset(&r, 0, sizeof(r));
      r.partial = partial + row;
      r.blocks = segment_blocks(n);
      r.ndots = seg.ndots;
      r.slot = reinterpret_cast<const int64_t*>(t + gb + pb) + seg.dot_slot0;
      r.red0 = red0;
      std::memcpy(host.data() + ro + k * sizeof(GroupRed), &r, sizeof(r));
      k++;
      red0 += seg.ndots;
    }
    row += segment_blocks(n) * seg.ndots;
  }
}

size_t segment_table_bytes(const SegmentPlan& P) {
  return segment_reds_offset(P) + P.segs.size() * sizeof(GroupRed) + 256;
}

void segment_table_host(const SegmentPlan& P, std::vector<char>& host, const std::vector<int64_t>& slots) {
  const size_t gb = ((P.gates.size() * sizeof(SegGate) + 255) / 256) * 256;
  const size_t pb = ((P.pool.size() * sizeof(double) + 255) / 256) * 256;
  host.assign(segment_table_bytes(P), 0);
  if (!P.gates.empty()) std::memcpy(host.data(), P.gates.data(), P.gates.size() * sizeof(SegGate));
  if (!P.pool.empty()) std::memcpy(host.data() + gb, P.pool.data(), P.pool.size() * sizeof(double));
  if (!slots.empty()) std::memcpy(host.data() + gb + pb, slots.data(), slots.size() * sizeof(int64_t));
}

size_t segment_pool_offset(const SegmentPlan& P) {
  return ((P.gates.size() * sizeof(SegGate) + 255) / 256) * 256;
}

int64_t segment_blocks(int n) {
  const int64_t ncos = (int64_t(1) << n) >> 3;
  return (ncos + kSegBlock - 1) / kSegBlock;
}


// ---------------------------------------------------------------------------
// Grouped sweeps: step k runs segment k of every plan that has one, for all
// states in one launch (and their dot sums in a second).
// ---------------------------------------------------------------------------

diaq_status_t build_grouped(const std::vector<GroupItem>& items, bool forward, GroupedSweep* out) {
  GroupedSweep& G = *out;
  G = GroupedSweep();
  G.forward = forward;
  size_t nsteps = 0;
  for (const auto& it : items) nsteps = std::max(nsteps, it.plan->segs.size());
  std::vector<GroupSeg> segs;
  std::vector<GroupRed> reds;
  for (size_t k = 0; k < nsteps; k++) {
    GroupedStep st;
    st.seg_first = int64_t(segs.size());
    st.red_first = int64_t(reds.size());
    int64_t blocks = 0, red_blocks = 0;
    for (const auto& it : items) {
      const SegmentPlan& P = *it.plan;
      if (k >= P.segs.size()) continue;
      const Segment& seg = P.segs[k];
      const char* t = static_cast<const char*>(it.table);
      const size_t gb = ((P.gates.size() * sizeof(SegGate) + 255) / 256) * 256;
      const size_t pb = ((P.pool.size() * sizeof(double) + 255) / 256) * 256;
      GroupSeg g;
      std::memset(&g, 0, sizeof(g));
      g.a = make_seg_args(P, seg, it.n, reinterpret_cast<const SegGate*>(t), reinterpret_cast<const double*>(t + gb));
      g.psi = it.psi;
      g.lam = it.lam;
      g.partial = it.partial;
      g.block0 = blocks;
      blocks += segment_blocks(it.n);
      segs.push_back(g);
      st.three = st.three || seg.three;
      if (!forward && seg.ndots) {
        GroupRed r;
        std::memset(&r, 0, sizeof(r));
        r.partial = it.partial;
        r.blocks = segment_blocks(it.n);
        r.ndots = seg.ndots;
        r.slot = reinterpret_cast<const int64_t*>(t + gb + pb) + seg.dot_slot0;
        r.red0 = red_blocks;
        red_blocks += seg.ndots;
        reds.push_back(r);
      }
    }
    st.seg_count = int64_t(segs.size()) - st.seg_first;
    st.red_count = int64_t(reds.size()) - st.red_first;
    st.blocks = blocks;
    st.red_blocks = red_blocks;
    if (blocks > 0x7fffffffLL) return fail(DIAQ_ERR_UNSUPPORTED, "grouped step needs %lld workgroups", (long long)blocks);
    G.steps.push_back(st);
  }
  const size_t sb = ((segs.size() * sizeof(GroupSeg) + 255) / 256) * 256;
  G.red_offset = sb;
  G.host.assign(sb + reds.size() * sizeof(GroupRed) + 256, 0);
  if (!segs.empty()) std::memcpy(G.host.data(), segs.data(), segs.size() * sizeof(GroupSeg));
  if (!reds.empty()) std::memcpy(G.host.data() + sb, reds.data(), reds.size() * sizeof(GroupRed));
  return DIAQ_OK;
}

diaq_status_t run_grouped(hipStream_t stream, const GroupedSweep& G, double* dots) {
  const GroupSeg* segs = static_cast<const GroupSeg*>(G.dev);
  const GroupRed* reds = reinterpret_cast<const GroupRed*>(static_cast<const char*>(G.dev) + G.red_offset);
  for (const GroupedStep& st : G.steps) {
    if (!st.seg_count) continue;
    const dim3 grid(unsigned(st.blocks)), block(kSegBlock);
    const GroupSeg* l = segs + st.seg_first;
    const int cnt = int(st.seg_count);
    if (G.forward) {
      if (st.three) hipLaunchKernelGGL((grouped_segment_kernel<double, false, true>), grid, block, 0, stream, l, cnt);
      else hipLaunchKernelGGL((grouped_segment_kernel<double, false, false>), grid, block, 0, stream, l, cnt);
    } else {
      if (st.three) hipLaunchKernelGGL((grouped_segment_kernel<double, true, true>), grid, block, 0, stream, l, cnt);
      else hipLaunchKernelGGL((grouped_segment_kernel<double, true, false>), grid, block, 0, stream, l, cnt);
    }
    DIAQ_HIP(hipGetLastError());
    if (st.red_count) {
      hipLaunchKernelGGL(grouped_reduce_kernel, dim3(unsigned(st.red_blocks)), dim3(256), 0, stream,
                         reds + st.red_first, int(st.red_count), dots);
      DIAQ_HIP(hipGetLastError());
    }
  }
  return DIAQ_OK;
}

}  // namespace diaq

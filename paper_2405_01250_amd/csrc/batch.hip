// batch.hip -- many small circuits of uneven width in one persistent launch.
//
// Each workgroup takes whole circuits from a device queue (an atomic
// counter over a host-sorted list, largest work first) until the queue is
// empty, so there is no inter-workgroup synchronisation and every wave
// reaches the exit.  Within a circuit the workgroup runs the forward pass,
// the diagonal observable, and the adjoint reverse sweep, gate by gate with
// workgroup barriers in between.  A gate is applied as Alg. 3 does it: its
// small local matrix acts on each coset of amplitudes that differ only in
// the gate's target bits (the rep x j loops of Alg. 3 enumerate exactly
// these cosets), in place, without expanding the 2^n matrix.  Circuits of
// at most 12 qubits keep both vectors (psi, lambda) in LDS (2 x 64 KiB);
// wider ones use per-circuit device buffers that stay in L2 / the 256 MB
// last-level cache for the widths of interest.
#include <algorithm>
#include <numeric>

#include "internal.hpp"

struct diaq_batch;

namespace diaq {

namespace {

constexpr int kThreads = 1024;
constexpr int kLdsMaxQubits = 12;

enum Rot : int32_t { kFixed = 0, kRX = 1, kRY = 2, kRZ = 3, kP = 4, kRXX = 5, kRYY = 6, kRZZ = 7 };

struct BGate {
  int32_t k, nc;
  int32_t q[2];   // targets, q[0] = local bit 0
  int32_t c[2];   // controls
  int32_t rot;    // rotation kind for angles taken from theta
  int32_t pidx;   // gradient slot within the circuit, -1 if none
  int32_t diag;   // diagonal local matrix
  int32_t pad;
  double scale;
  int64_t p0;          // the circuit's first parameter slot
  double m[4][4][2];   // local matrix at params[0]
  double g[4][4][2];   // generator (differentiable gates)
};

struct BCirc {
  int32_t n, nparams;
  int64_t g0, ng;   // gate range
  int64_t t0;       // observable term range
  int32_t nt, lds;  // number of terms; 1 = vectors in LDS
  int64_t p0;       // first parameter / gradient slot
  int64_t s0;       // workspace offset (elements) of psi; lambda follows
};

struct BatchArgs {
  const BCirc* circ;
  const BGate* gates;
  const uint64_t* zmask;
  const double* coef;
  const double* theta;  // device, may be null
  const double* mats;   // device, 32 doubles per gate: matrices at theta
  const int32_t* order;
  int32_t ncirc;
  int32_t use_theta;
  double2* ws;
  double* expvals;
  double* grads;
  int32_t* queue;
};

__device__ __forceinline__ void rot_matrix(int rot, double a, double m[4][4][2]) {
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 4; c++) m[r][c][0] = m[r][c][1] = 0.0;
  double s, c;
  sincos(0.5 * a, &s, &c);
  switch (rot) {
    case kRX:
      m[0][0][0] = c; m[1][1][0] = c; m[0][1][1] = -s; m[1][0][1] = -s;
      break;
    case kRY:
      m[0][0][0] = c; m[1][1][0] = c; m[0][1][0] = -s; m[1][0][0] = s;
      break;
    case kRZ:
      m[0][0][0] = c; m[0][0][1] = -s; m[1][1][0] = c; m[1][1][1] = s;
      break;
    case kP: {
      double s2, c2;
      sincos(a, &s2, &c2);
      m[0][0][0] = 1.0; m[1][1][0] = c2; m[1][1][1] = s2;
      break;
    }
    case kRXX:
      for (int r = 0; r < 4; r++) {
        m[r][r][0] = c;
        m[r][r ^ 3][1] = -s;
      }
      break;
    case kRYY:
      // Y(x)Y: -1 on the 00<->11 pair, +1 on the 01<->10 pair
      for (int r = 0; r < 4; r++) {
        m[r][r][0] = c;
        const double yy = (r == 0 || r == 3) ? -1.0 : 1.0;
        m[r][r ^ 3][1] = -s * yy;
      }
      break;
    case kRZZ:
      for (int r = 0; r < 4; r++) {
        const bool odd = ((r & 1) ^ (r >> 1)) != 0;
        m[r][r][0] = c;
        m[r][r][1] = odd ? s : -s;
      }
      break;
    default:
      break;
  }
}

__device__ __forceinline__ int64_t coset_base(int64_t cb, const BGate& g) {
  int p0 = g.q[0], p1 = g.k > 1 ? g.q[1] : 64;
  if (p1 < p0) {
    const int t = p0;
    p0 = p1;
    p1 = t;
  }
  int64_t b = (cb & ((int64_t(1) << p0) - 1)) | ((cb >> p0) << (p0 + 1));
  if (g.k > 1) b = (b & ((int64_t(1) << p1) - 1)) | ((b >> p1) << (p1 + 1));
  return b;
}

__device__ __forceinline__ bool controls_ok(int64_t b, const BGate& g) {
  for (int j = 0; j < g.nc; j++)
    if (!((b >> g.c[j]) & 1)) return false;
  return true;
}

__device__ __forceinline__ int64_t local_offset(int r, const BGate& g) {
  int64_t o = 0;
  for (int j = 0; j < g.k; j++)
    if ((r >> j) & 1) o |= int64_t(1) << g.q[j];
  return o;
}

// v <- M v (or M^dagger v) on every coset whose controls are 1.  K is the
// number of targets, so every local index below is a compile-time constant.
template <int K>
__device__ void apply_gate(double2* v, int n, const BGate& g, const double (*m)[4][2], bool adjoint) {
  constexpr int d = 1 << K;
  const int64_t ncos = (int64_t(1) << n) >> K;
  for (int64_t cb = threadIdx.x; cb < ncos; cb += kThreads) {
    __asm__ volatile("" ::: "memory");  // keep the staged matrix in LDS
    const int64_t b = coset_base(cb, g);
    if (!controls_ok(b, g)) continue;
    double2 a[d];
#pragma unroll
    for (int r = 0; r < d; r++) a[r] = v[b + local_offset(r, g)];
#pragma unroll
    for (int r = 0; r < d; r++) {
      double xr = 0, xi = 0;
#pragma unroll
      for (int c = 0; c < d; c++) {
        const double mr = adjoint ? m[c][r][0] : m[r][c][0];
        const double mi = adjoint ? -m[c][r][1] : m[r][c][1];
        xr += mr * a[c].x - mi * a[c].y;
        xi += mr * a[c].y + mi * a[c].x;
      }
      v[b + local_offset(r, g)] = double2{xr, xi};
    }
  }
}

// sum over cosets with controls 1 of conj(lam) (G psi); per-lane partial.
template <int K>
__device__ double2 gen_dot(const double2* lam, const double2* psi, int n, const BGate& g,
                        const double (*gm)[4][2]) {
  constexpr int d = 1 << K;
  const int64_t ncos = (int64_t(1) << n) >> K;
  double re = 0, im = 0;
  for (int64_t cb = threadIdx.x; cb < ncos; cb += kThreads) {
    // compiler barrier: re-read the staged matrix from LDS each iteration
    // instead of pinning 32 doubles in registers
    __asm__ volatile("" ::: "memory");
    const int64_t b = coset_base(cb, g);
    if (!controls_ok(b, g)) continue;
    double2 a[d];
#pragma unroll
    for (int r = 0; r < d; r++) a[r] = psi[b + local_offset(r, g)];
#pragma unroll
    for (int r = 0; r < d; r++) {
      double gr = 0, gi = 0;
#pragma unroll
      for (int c = 0; c < d; c++) {
        gr += gm[r][c][0] * a[c].x - gm[r][c][1] * a[c].y;
        gi += gm[r][c][0] * a[c].y + gm[r][c][1] * a[c].x;
      }
      const double2 l = lam[b + local_offset(r, g)];
      re += l.x * gr + l.y * gi;
      im += l.x * gi - l.y * gr;
    }
  }
  return double2{re, im};
}

// Fixed-order workgroup sum; every thread gets the result.
__device__ double2 wg_sum(double2 v, double2* wsum) {
  for (int off = 32; off >= 1; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wsum[wave] = v;
  __syncthreads();
  double2 t = wsum[0];
  for (int w = 1; w < kThreads / 64; w++) {
    t.x += wsum[w].x;
    t.y += wsum[w].y;
  }
  __syncthreads();
  return t;
}

// Copy a 4 x 4 complex matrix (32 doubles) into LDS, one double per lane.
__device__ __forceinline__ void stage_matrix(const double* src, double (&dst)[4][4][2]) {
  if (threadIdx.x < 32) (&dst[0][0][0])[threadIdx.x] = src[threadIdx.x];
}

__device__ __forceinline__ const double* gate_matrix(const BatchArgs& a, int64_t gidx, const BGate& g) {
  return (a.use_theta && g.pidx >= 0 && g.rot != kFixed) ? a.mats + gidx * 32 : &g.m[0][0][0];
}

// Angles from theta: the local matrix of every differentiable rotation (one
// lane per gate), written to a side table before the batch kernel runs.
__global__ void batch_angles_kernel(const BGate* gates, int64_t ngates, const double* theta, double* mats) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ngates) return;
  const BGate& g = gates[i];
  if (g.pidx < 0 || g.rot == kFixed) return;
  double m[4][4][2];
  rot_matrix(g.rot, g.scale * theta[g.p0 + g.pidx], m);
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 4; c++) {
      mats[i * 32 + (r * 4 + c) * 2] = m[r][c][0];
      mats[i * 32 + (r * 4 + c) * 2 + 1] = m[r][c][1];
    }
}

__global__ __launch_bounds__(kThreads) void batch_kernel(BatchArgs a) {
  extern __shared__ double2 lds[];
  __shared__ double2 wsum[kThreads / 64];
  __shared__ int s_item;
  // the current gate's local matrix and generator, staged in LDS
  __shared__ double sm[4][4][2];
  __shared__ double sg[4][4][2];
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= a.ncirc) break;
    const BCirc cc = a.circ[a.order[item]];
    const int n = cc.n;
    const int64_t N = int64_t(1) << n;
    double2* psi = cc.lds ? lds : a.ws + cc.s0;
    double2* lam = cc.lds ? lds + (int64_t(1) << kLdsMaxQubits) : a.ws + cc.s0 + N;
    for (int64_t i = threadIdx.x; i < N; i += kThreads) psi[i] = double2{i == 0 ? 1.0 : 0.0, 0.0};
    __syncthreads();
    // forward
    for (int64_t gi = 0; gi < cc.ng; gi++) {
      const BGate& g = a.gates[cc.g0 + gi];
      stage_matrix(gate_matrix(a, cc.g0 + gi, g), sm);
      __syncthreads();
      if (g.k == 1) apply_gate<1>(psi, n, g, sm, false);
      else apply_gate<2>(psi, n, g, sm, false);
      __syncthreads();
    }
    // lambda = H psi (H diagonal), E = <psi|lambda>
    double2 acc{0, 0};
    for (int64_t i = threadIdx.x; i < N; i += kThreads) {
      double h = 0;
      for (int t = 0; t < cc.nt; t++)
        h += (__popcll(uint64_t(i) & a.zmask[cc.t0 + t]) & 1) ? -a.coef[cc.t0 + t] : a.coef[cc.t0 + t];
      const double2 p = psi[i];
      const double2 l{h * p.x, h * p.y};
      lam[i] = l;
      acc.x += p.x * l.x + p.y * l.y;
      acc.y += p.x * l.y - p.y * l.x;
    }
    const double2 e = wg_sum(acc, wsum);
    if (threadIdx.x == 0) a.expvals[a.order[item]] = e.x;
    // reverse sweep
    for (int64_t gi = cc.ng - 1; gi >= 0; gi--) {
      const BGate& g = a.gates[cc.g0 + gi];
      if (g.pidx >= 0) {
        stage_matrix(&g.g[0][0][0], sg);
        __syncthreads();
        const double2 part = g.k == 1 ? gen_dot<1>(lam, psi, n, g, sg) : gen_dot<2>(lam, psi, n, g, sg);
        const double2 dsum = wg_sum(part, wsum);
        if (threadIdx.x == 0) a.grads[cc.p0 + g.pidx] += g.scale * dsum.y;
      }
      if (gi == 0) break;
      stage_matrix(gate_matrix(a, cc.g0 + gi, g), sm);
      __syncthreads();
      if (g.k == 1) {
        apply_gate<1>(psi, n, g, sm, true);
        apply_gate<1>(lam, n, g, sm, true);
      } else {
        apply_gate<2>(psi, n, g, sm, true);
        apply_gate<2>(lam, n, g, sm, true);
      }
      __syncthreads();
    }
    __syncthreads();
  }
}

__global__ void batch_reset_kernel(int32_t* queue, double* expvals, int64_t nc, double* grads, int64_t ng) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i == 0) *queue = 0;
  if (i < nc) expvals[i] = 0.0;
  if (i < ng) grads[i] = 0.0;
}
// ---------------------------------------------------------------------------
// Wide circuits (too large for one workgroup): all of them advance together.
// Each step is one launch whose grid is the concatenation of every wide
// circuit's workgroups (segment passes of the segmented Alg. 3 sweep, the
// observable, the initial state), so a few dozen launches cover the lot and
// the GPU is full even when each state alone would occupy a few CUs.
// ---------------------------------------------------------------------------

constexpr int kWideMinQubits = 15;
constexpr int kSideStreams = 1;  // the persistent kernel runs beside the wide steps
constexpr int kObsBlock = 256;
// amplitudes per lane in the grouped init / observable grids: enough work per
// workgroup to amortise the search for its circuit (N >= 2^15 is a multiple
// of the 4096 amplitudes a workgroup covers)
constexpr int kObsPerLane = 16;
constexpr int64_t kObsSpan = int64_t(kObsBlock) * kObsPerLane;

// One wide circuit's vectors for the grouped init / observable kernels.
struct WideVec {
  double2* psi;
  double2* lam;
  int64_t N;
  const uint64_t* zm;
  const double* coef;
  int32_t nt;
  int32_t pad;
  double2* partial;
  double2* eval;
  int64_t block0;  // first workgroup of this circuit in the grouped grid (N / kObsSpan each)
};

__device__ __forceinline__ int find_item(const WideVec* __restrict__ list, int count) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (list[mid].block0 <= int64_t(blockIdx.x)) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kObsBlock) void grouped_init_kernel(const WideVec* __restrict__ list, int count) {
  using ND = Nat<double>::T;
  const WideVec& w = list[find_item(list, count)];
  const int64_t i0 = (int64_t(blockIdx.x) - w.block0) * kObsSpan + threadIdx.x;
  auto* psi = gptr(reinterpret_cast<ND*>(w.psi));
#pragma unroll
  for (int e = 0; e < kObsPerLane; e++) {
    const int64_t i = i0 + int64_t(e) * kObsBlock;
    if (i < w.N) psi[i] = ND{i == 0 ? 1.0 : 0.0, 0.0};
  }
}

// lambda = H psi for the diagonal observable; one partial <psi|lambda> per
// workgroup.  A lane's amplitudes are loaded first, then each term is read
// once (scalar loads: the term tables are constant while the kernel runs)
// and applied to all of them.
__global__ __launch_bounds__(kObsBlock) void grouped_observable_kernel(const WideVec* __restrict__ list, int count) {
  using ND = Nat<double>::T;
  typedef __attribute__((address_space(4))) const uint64_t CU64;
  typedef __attribute__((address_space(4))) const double CDouble;
  const WideVec& w = list[find_item(list, count)];
  const int64_t blk = int64_t(blockIdx.x) - w.block0;
  const auto* __restrict__ psi = gptr(reinterpret_cast<const ND*>(w.psi));
  auto* __restrict__ lam = gptr(reinterpret_cast<ND*>(w.lam));
  CU64* zm = (CU64*)(w.zm);
  CDouble* coef = (CDouble*)(w.coef);
  const int64_t N = w.N;
  const int nt = w.nt;
  const int64_t i0 = blk * kObsSpan + threadIdx.x;
  ND p[kObsPerLane];
  double h[kObsPerLane];
#pragma unroll
  for (int e = 0; e < kObsPerLane; e++) {
    const int64_t i = i0 + int64_t(e) * kObsBlock;
    p[e] = i < N ? psi[i] : ND{0, 0};
    h[e] = 0;
  }
  for (int t = 0; t < nt; t++) {
    const uint64_t z = zm[t];
    const double c = coef[t];
#pragma unroll
    for (int e = 0; e < kObsPerLane; e++)
      h[e] += (__popcll(uint64_t(i0 + int64_t(e) * kObsBlock) & z) & 1) ? -c : c;
  }
  double re = 0, im = 0;
#pragma unroll
  for (int e = 0; e < kObsPerLane; e++) {
    const int64_t i = i0 + int64_t(e) * kObsBlock;
    if (i >= N) break;
    const ND l{h[e] * p[e].x, h[e] * p[e].y};
    lam[i] = l;
    re += p[e].x * l.x + p[e].y * l.y;
    im += p[e].x * l.y - p[e].y * l.x;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  __shared__ double2 wsum[kObsBlock / 64];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = double2{re, im};
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 t = wsum[0];
    for (int q = 1; q < kObsBlock / 64; q++) {
      t.x += wsum[q].x;
      t.y += wsum[q].y;
    }
    gptr(reinterpret_cast<ND*>(w.partial))[blk] = ND{t.x, t.y};
  }
}

// E of every wide circuit: workgroup c sums circuit c's observable partials
// in a fixed order.
__global__ __launch_bounds__(256) void grouped_eval_kernel(const WideVec* __restrict__ list) {
  const WideVec& w = list[blockIdx.x];
  const int64_t nb = (w.N + kObsSpan - 1) / kObsSpan;
  const auto* part = gptr(reinterpret_cast<const Nat<double>::T*>(w.partial));
  double re = 0, im = 0;
  for (int64_t b = threadIdx.x; b < nb; b += 256) {
    const auto v = part[b];
    re += v.x;
    im += v.y;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  __shared__ double2 ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = double2{re, im};
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 t = ws[0];
    for (int q = 1; q < 4; q++) {
      t.x += ws[q].x;
      t.y += ws[q].y;
    }
    gptr(reinterpret_cast<Nat<double>::T*>(w.eval))[0] = Nat<double>::T{t.x, t.y};
  }
}

struct WideRes {
  int32_t circ;
  int32_t ndots;
  int64_t dot0;  // first slot in the dot table
  int64_t p0;    // first gradient slot of the circuit
};

struct WideDot {
  int32_t pidx;
  int32_t pad;
  double scale;
};

// One lane per wide circuit: expectation value and gradient sums in a fixed
// (reverse-sweep) order.
__global__ void wide_finalize_kernel(const WideRes* __restrict__ res, int nwide, const WideDot* __restrict__ meta,
                                     const double2* __restrict__ dots, const double2* __restrict__ evals,
                                     double* __restrict__ expvals, double* __restrict__ grads) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwide) return;
  const WideRes r = res[w];
  expvals[r.circ] = evals[w].x;
  for (int j = 0; j < r.ndots; j++) grads[r.p0 + meta[r.dot0 + j].pidx] += meta[r.dot0 + j].scale * dots[r.dot0 + j].y;
}

int rot_of(int kind) {
  switch (kind) {
    case DIAQ_GATE_RX: return kRX;
    case DIAQ_GATE_RY: return kRY;
    case DIAQ_GATE_RZ: return kRZ;
    case DIAQ_GATE_P: return kP;
    case DIAQ_GATE_RXX: return kRXX;
    case DIAQ_GATE_RYY: return kRYY;
    case DIAQ_GATE_RZZ: return kRZZ;
    default: return kFixed;
  }
}

struct WideCirc {
  int32_t c = 0, n = 0;
  int64_t g0 = 0;    // first gate in the batch gate table
  int64_t s0 = 0;    // workspace offset of psi (lambda follows)
  int64_t t0 = 0;    // first observable term
  int32_t nt = 0;
  int64_t dot0 = 0;  // first dot slot
  std::vector<LocalGate> lg, gen;
  std::vector<int32_t> pidx, rot;
  std::vector<double> angle0;  // each gate's own angle (params[0])
  std::vector<double> scale;
  SegmentPlan fwd, rev;        // forward pass and reverse sweep, several gates per pass
  size_t o_fwd = 0, o_rev = 0; // their device tables, offsets into the batch block
  size_t o_part = 0;           // this circuit's partial sums (offset into the partial region)
  int64_t npart = 0;           // entries
  void* d_fwd = nullptr;
  void* d_rev = nullptr;
};

// A rotation whose matrix sits in a segment table: rewritten from the angle
// before each run (the angle from theta, or the gate's own angle).
struct SegPatch {
  double* dst;
  int32_t rot;
  int32_t diag;    // 1: the table holds the diagonal only
  int32_t dim;     // 2 or 4
  int32_t dagger;  // 1: store U^dagger (reverse sweep)
  int64_t slot;    // theta index
  double scale;
  double angle0;
};

__global__ void seg_patch_kernel(const SegPatch* __restrict__ patches, int64_t count,
                                 const double* __restrict__ theta) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const SegPatch p = patches[i];
  double m[4][4][2];
  rot_matrix(p.rot, theta ? p.scale * theta[p.slot] : p.angle0, m);
  const double sg = p.dagger ? -1.0 : 1.0;
  if (p.diag) {
    for (int r = 0; r < p.dim; r++) {
      p.dst[2 * r] = m[r][r][0];
      p.dst[2 * r + 1] = sg * m[r][r][1];
    }
  } else {
    for (int r = 0; r < p.dim; r++)
      for (int c = 0; c < p.dim; c++) {
        const int rr = p.dagger ? c : r, cc = p.dagger ? r : c;
        p.dst[2 * (r * p.dim + c)] = m[rr][cc][0];
        p.dst[2 * (r * p.dim + c) + 1] = sg * m[rr][cc][1];
      }
  }
}

}  // namespace
}  // namespace diaq

struct diaq_batch {
  diaq_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t side[diaq::kSideStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[diaq::kSideStreams] = {};
  int32_t ncirc = 0;
  int32_t nnarrow = 0;
  int64_t nparams = 0;
  int64_t ngates = 0;
  void* dmem = nullptr;          // tables, results, queue, partials
  double2* ws = nullptr;         // per-circuit vectors outside LDS
  diaq::BatchArgs args{};
  std::vector<diaq::WideCirc> wide;
  diaq::WideRes* d_wres = nullptr;
  diaq::WideDot* d_wmeta = nullptr;
  double2* d_dots = nullptr;
  double2* d_evals = nullptr;
  void* gmem = nullptr;          // grouped-launch descriptors
  diaq::GroupedSweep gfwd, grev;
  diaq::WideVec* d_wvec = nullptr;
  int64_t wblocks = 0;           // workgroups of the grouped init / observable grids
  diaq::SegPatch* d_patch = nullptr;
  int64_t npatch = 0;
  double* pinned = nullptr;      // theta in, expvals + grads out
  int64_t pinned_theta = 0, pinned_out = 0;
  size_t lds_bytes = 0;
  int grid = 0;
  bool graph = false;
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  bool have_theta_graph = false;
};

namespace diaq {
namespace {

diaq_status_t enqueue(diaq_batch* b, bool use_theta) {
  BatchArgs args = b->args;
  args.use_theta = use_theta ? 1 : 0;
  if (use_theta) {
    DIAQ_HIP(hipMemcpyAsync(const_cast<double*>(args.theta), b->pinned, size_t(b->nparams) * sizeof(double),
                            hipMemcpyHostToDevice, b->stream));
    if (b->ngates)
      hipLaunchKernelGGL(batch_angles_kernel, dim3(unsigned((b->ngates + 255) / 256)), dim3(256), 0, b->stream,
                         args.gates, b->ngates, args.theta, const_cast<double*>(args.mats));
    DIAQ_HIP(hipGetLastError());
  }
  const int64_t nz = std::max<int64_t>(std::max<int64_t>(b->ncirc, b->nparams), 1);
  hipLaunchKernelGGL(batch_reset_kernel, dim3(unsigned((nz + 255) / 256)), dim3(256), 0, b->stream, args.queue,
                     args.expvals, int64_t(b->ncirc), args.grads, b->nparams);
  DIAQ_HIP(hipGetLastError());
  const bool wide = !b->wide.empty();
  if (b->npatch) {
    hipLaunchKernelGGL(seg_patch_kernel, dim3(unsigned((b->npatch + 255) / 256)), dim3(256), 0, b->stream, b->d_patch,
                       b->npatch, use_theta ? args.theta : nullptr);
    DIAQ_HIP(hipGetLastError());
  }
  // the persistent kernel runs on the side stream while the wide circuits
  // step together on the batch stream
  const bool side = wide && b->nnarrow;
  if (side) {
    DIAQ_HIP(hipEventRecord(b->fork, b->stream));
    DIAQ_HIP(hipStreamWaitEvent(b->side[0], b->fork, 0));
  }
  if (b->nnarrow) {
    hipLaunchKernelGGL(batch_kernel, dim3(unsigned(b->grid)), dim3(kThreads), b->lds_bytes,
                       side ? b->side[0] : b->stream, args);
    DIAQ_HIP(hipGetLastError());
  }
  if (wide) {
    const int nw = int(b->wide.size());
    hipLaunchKernelGGL(grouped_init_kernel, dim3(unsigned(b->wblocks)), dim3(kObsBlock), 0, b->stream, b->d_wvec, nw);
    DIAQ_HIP(hipGetLastError());
    DIAQ_TRY(run_grouped(b->stream, b->gfwd, nullptr));
    hipLaunchKernelGGL(grouped_observable_kernel, dim3(unsigned(b->wblocks)), dim3(kObsBlock), 0, b->stream,
                       b->d_wvec, nw);
    DIAQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(grouped_eval_kernel, dim3(unsigned(nw)), dim3(256), 0, b->stream, b->d_wvec);
    DIAQ_HIP(hipGetLastError());
    DIAQ_TRY(run_grouped(b->stream, b->grev, reinterpret_cast<double*>(b->d_dots)));
    hipLaunchKernelGGL(wide_finalize_kernel, dim3(unsigned((nw + 63) / 64)), dim3(64), 0, b->stream, b->d_wres, nw,
                       b->d_wmeta, b->d_dots, b->d_evals, args.expvals, args.grads);
    DIAQ_HIP(hipGetLastError());
  }
  if (side) {
    DIAQ_HIP(hipEventRecord(b->join[0], b->side[0]));
    DIAQ_HIP(hipStreamWaitEvent(b->stream, b->join[0], 0));
  }
  double* out = b->pinned + b->pinned_theta;
  DIAQ_HIP(hipMemcpyAsync(out, args.expvals, size_t(b->ncirc) * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  if (b->nparams)
    DIAQ_HIP(hipMemcpyAsync(out + b->ncirc, args.grads, size_t(b->nparams) * sizeof(double), hipMemcpyDeviceToHost,
                            b->stream));
  return DIAQ_OK;
}

}  // namespace
}  // namespace diaq

using namespace diaq;

extern "C" {

diaq_status_t diaq_batch_free(diaq_batch_t b) {
  if (!b) return DIAQ_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (int j = 0; j < kSideStreams; j++)
    if (b->side[j]) (void)hipStreamSynchronize(b->side[j]);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->g) (void)hipGraphDestroy(b->g);
  if (b->dmem) (void)hipFree(b->dmem);
  if (b->gmem) (void)hipFree(b->gmem);
  if (b->ws) (void)hipFree(b->ws);
  if (b->pinned) (void)hipHostFree(b->pinned);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (int j = 0; j < kSideStreams; j++) {
    if (b->join[j]) (void)hipEventDestroy(b->join[j]);
    if (b->side[j]) (void)hipStreamDestroy(b->side[j]);
  }
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return DIAQ_OK;
}

diaq_status_t diaq_batch_create(diaq_ctx_t ctx, const diaq_circuit_t* circuits, int32_t ncircuits, uint32_t flags,
                                diaq_batch_t* out) {
  try {
    if (!ctx || !out || ncircuits < 0 || (ncircuits > 0 && !circuits))
      return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad batch arguments");
    if (flags & ~DIAQ_BATCH_GRAPH) return fail(DIAQ_ERR_INVALID_ARGUMENT, "unknown batch flags 0x%x", flags);
    std::vector<BCirc> circ(static_cast<size_t>(ncircuits));
    std::vector<BGate> gates;
    std::vector<uint64_t> zm;
    std::vector<double> coef;
    std::vector<WideCirc> wide;
    std::vector<WideRes> wres;
    std::vector<WideDot> wmeta;
    int64_t nparams = 0, ws_elems = 0;
    std::vector<double> work(static_cast<size_t>(ncircuits));
    std::vector<int32_t> narrow;
    for (int c = 0; c < ncircuits; c++) {
      const diaq_circuit_t& C = circuits[c];
      if (C.nqubits < 1 || C.nqubits > 30) return fail(DIAQ_ERR_INVALID_ARGUMENT, "circuit %d: nqubits %d", c, C.nqubits);
      if (C.ngates < 0 || (C.ngates > 0 && !C.gates) || C.nparams < 0 || C.nterms < 0 ||
          (C.nterms > 0 && (!C.zmask || !C.coef)))
        return fail(DIAQ_ERR_INVALID_ARGUMENT, "circuit %d: bad arrays", c);
      const bool is_wide = C.nqubits >= kWideMinQubits;
      BCirc& bc = circ[c];
      bc.n = C.nqubits;
      bc.nparams = C.nparams;
      bc.g0 = int64_t(gates.size());
      bc.ng = C.ngates;
      bc.t0 = int64_t(zm.size());
      bc.nt = C.nterms;
      bc.p0 = nparams;
      bc.lds = C.nqubits <= kLdsMaxQubits ? 1 : 0;
      bc.s0 = bc.lds ? -1 : ws_elems;
      if (!bc.lds) ws_elems += 2 * (int64_t(1) << C.nqubits);
      nparams += C.nparams;
      for (int t = 0; t < C.nterms; t++) {
        if (C.zmask[t] >> C.nqubits) return fail(DIAQ_ERR_INVALID_ARGUMENT, "circuit %d: term %d outside register", c, t);
        zm.push_back(C.zmask[t]);
        coef.push_back(C.coef[t]);
      }
      WideCirc wc;
      if (is_wide) {
        wc.c = c;
        wc.n = C.nqubits;
        wc.g0 = bc.g0;
        wc.s0 = bc.s0;
        wc.t0 = bc.t0;
        wc.nt = bc.nt;
      }
      for (int64_t gi = 0; gi < C.ngates; gi++) {
        const diaq_gate_t* g = &C.gates[gi];
        LocalGate lg;
        diaq_status_t st = local_gate(g, C.nqubits, &lg);
        if (st != DIAQ_OK) return fail(st, "circuit %d gate %lld: %s", c, (long long)gi, diaq_last_error());
        if (lg.k > 2 || lg.nc > 2)
          return fail(DIAQ_ERR_UNSUPPORTED, "circuit %d gate %lld: batched gates take <= 2 targets and <= 2 controls",
                      c, (long long)gi);
        BGate bg;
        std::memset(&bg, 0, sizeof(bg));
        bg.k = lg.k;
        bg.nc = lg.nc;
        for (int j = 0; j < lg.k; j++) bg.q[j] = lg.targets[j];
        for (int j = 0; j < lg.nc; j++) bg.c[j] = lg.controls[j];
        const int d = 1 << lg.k;
        bool diag = true;
        for (int r = 0; r < d; r++)
          for (int cc = 0; cc < d; cc++) {
            bg.m[r][cc][0] = lg.m[r][cc][0];
            bg.m[r][cc][1] = lg.m[r][cc][1];
            if (r != cc && lg.structural[r][cc]) diag = false;
          }
        bg.diag = diag ? 1 : 0;
        bg.rot = rot_of(g->kind);
        bg.pidx = -1;
        LocalGate gen = lg;
        if (g->param_index >= 0) {
          if (g->param_index >= C.nparams)
            return fail(DIAQ_ERR_INVALID_ARGUMENT, "circuit %d gate %lld: param_index out of range", c, (long long)gi);
          if (!local_generator(g, &gen))
            return fail(DIAQ_ERR_UNSUPPORTED, "circuit %d gate %lld: not a rotation", c, (long long)gi);
          for (int r = 0; r < d; r++)
            for (int cc = 0; cc < d; cc++) {
              bg.g[r][cc][0] = gen.m[r][cc][0];
              bg.g[r][cc][1] = gen.m[r][cc][1];
            }
          bg.pidx = g->param_index;
          bg.scale = g->param_scale;
          bg.p0 = bc.p0;
        }
        gates.push_back(bg);
        if (is_wide) {
          wc.lg.push_back(lg);
          wc.gen.push_back(gen);
          wc.pidx.push_back(bg.pidx);
          wc.rot.push_back(bg.rot);
          wc.angle0.push_back(g->params[0]);
          wc.scale.push_back(g->param_scale);
        }
      }
      work[c] = double(int64_t(1) << C.nqubits) * double(3 * C.ngates + 1);
      if (is_wide) {
        WideRes r;
        r.circ = c;
        r.dot0 = int64_t(wmeta.size());
        r.p0 = bc.p0;
        wc.dot0 = r.dot0;
        // segment plans; dot slots in the reverse sweep's order (gates that
        // share a parameter and scale inside a diagonal run share a dot)
        std::vector<int64_t> dkey(wc.lg.size(), -1);
        for (size_t j = 0; j < wc.lg.size(); j++)
          if (wc.pidx[j] >= 0) {
            int64_t key = -1;
            for (size_t i2 = 0; i2 < j && key < 0; i2++)
              if (wc.pidx[i2] == wc.pidx[j] && wc.scale[i2] == wc.scale[j]) key = dkey[i2];
            dkey[j] = key >= 0 ? key : int64_t(j);
          }
        DIAQ_TRY(plan_segments(wc.lg, wc.gen, dkey, wc.n, &wc.fwd, true));
        DIAQ_TRY(plan_segments(wc.lg, wc.gen, dkey, wc.n, &wc.rev, false));
        for (int64_t gi : wc.rev.dot_gate)
          wmeta.push_back(WideDot{wc.pidx[size_t(gi)], 0, wc.scale[size_t(gi)]});
        r.ndots = int32_t(int64_t(wmeta.size()) - r.dot0);
        wres.push_back(r);
        wide.push_back(std::move(wc));
      } else {
        narrow.push_back(c);
      }
    }
    // narrow circuits: queue order, largest work first
    std::stable_sort(narrow.begin(), narrow.end(), [&](int32_t x, int32_t y) { return work[x] > work[y]; });
    size_t part_bytes = 0;
    size_t seg_bytes = 0;
    std::vector<std::vector<char>> seg_host;
    for (auto& w : wide) {
      // partial sums: the observable's, and the reverse sweep's per-segment dots
      int32_t maxdots = 1;
      for (const auto& sg : w.rev.segs) maxdots = std::max(maxdots, sg.ndots);
      w.npart = std::max<int64_t>(((int64_t(1) << w.n) + kObsSpan - 1) / kObsSpan, segment_blocks(w.n) * maxdots);
      w.o_part = part_bytes;
      part_bytes += (size_t(w.npart) * sizeof(double2) + 255) / 256 * 256;
      std::vector<int64_t> slots(w.rev.dot_gate.size());
      for (size_t j = 0; j < slots.size(); j++) slots[j] = w.dot0 + int64_t(j);
      seg_host.emplace_back();
      segment_table_host(w.fwd, seg_host.back(), {});
      w.o_fwd = seg_bytes;
      seg_bytes += (seg_host.back().size() + 255) / 256 * 256;
      seg_host.emplace_back();
      segment_table_host(w.rev, seg_host.back(), slots);
      w.o_rev = seg_bytes;
      seg_bytes += (seg_host.back().size() + 255) / 256 * 256;
    }

    diaq_batch* b = new diaq_batch();
    b->ctx = ctx;
    b->ncirc = ncircuits;
    b->nnarrow = int32_t(narrow.size());
    b->nparams = nparams;
    auto bail = [&](diaq_status_t st) {
      diaq_batch_free(b);
      return st;
    };
#define DIAQ_TRY_BAIL(expr)              \
  do {                                   \
    diaq_status_t s_ = (expr);           \
    if (s_ != DIAQ_OK) return bail(s_);  \
  } while (0)
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(DIAQ_ERR_DEVICE, "hipStreamCreate failed"));
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
      return bail(fail(DIAQ_ERR_DEVICE, "hipEventCreate failed"));
    for (int j = 0; j < kSideStreams; j++) {
      if (hipStreamCreateWithFlags(&b->side[j], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&b->join[j], hipEventDisableTiming) != hipSuccess)
        return bail(fail(DIAQ_ERR_DEVICE, "side stream setup failed"));
    }
    // one device block for every table
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t off = 0;
    const size_t o_circ = off; off += al(circ.size() * sizeof(BCirc) + 1);
    const size_t o_gates = off; off += al(gates.size() * sizeof(BGate) + 1);
    const size_t o_zm = off; off += al(zm.size() * sizeof(uint64_t) + 1);
    const size_t o_coef = off; off += al(coef.size() * sizeof(double) + 1);
    const size_t o_order = off; off += al(narrow.size() * sizeof(int32_t) + 1);
    const size_t o_theta = off; off += al(size_t(nparams) * sizeof(double) + 1);
    const size_t o_mats = off; off += al(gates.size() * 32 * sizeof(double) + 1);
    const size_t o_exp = off; off += al(size_t(ncircuits) * sizeof(double) + 1);
    const size_t o_grad = off; off += al(size_t(nparams) * sizeof(double) + 1);
    const size_t o_queue = off; off += 256;
    const size_t o_wres = off; off += al(wres.size() * sizeof(WideRes) + 1);
    const size_t o_wmeta = off; off += al(wmeta.size() * sizeof(WideDot) + 1);
    const size_t o_dots = off; off += al(wmeta.size() * sizeof(double2) + 1);
    const size_t o_evals = off; off += al(wide.size() * sizeof(double2) + 1);
    const size_t o_part = off; off += al(part_bytes + 1);
    const size_t o_seg = off; off += al(seg_bytes + 1);
    // matrices of rotations inside the segment tables
    std::vector<SegPatch> patches;
    for (const auto& w : wide)
      for (const SegmentPlan* P : {&w.fwd, &w.rev})
        for (size_t i = 0; i < P->gates.size(); i++) {
          const int64_t m = P->gate_of[i];
          if (w.pidx[size_t(m)] < 0 || w.rot[size_t(m)] == kFixed) continue;
          SegPatch sp;
          std::memset(&sp, 0, sizeof(sp));
          sp.rot = w.rot[size_t(m)];
          if (P->gates[i].kind == 4) continue;  // run header
          sp.diag = (P->gates[i].kind == 5 || P->gates[i].kind == 3) ? 1 : 0;
          sp.dim = sp.diag ? (1 << P->gates[i].dk) : (P->gates[i].kind == 0 ? 2 : 4);
          sp.dagger = P->forward ? 0 : 1;
          sp.slot = circ[size_t(w.c)].p0 + w.pidx[size_t(m)];
          sp.scale = w.scale[size_t(m)];
          sp.angle0 = w.angle0[size_t(m)];
          // device address, filled in below: table offset + pool offset + moff
          sp.dst = reinterpret_cast<double*>(
              (P == &w.fwd ? w.o_fwd : w.o_rev) + segment_pool_offset(*P) + size_t(P->gates[i].moff) * sizeof(double));
          patches.push_back(sp);
        }
    const size_t o_patch = off; off += al(patches.size() * sizeof(SegPatch) + 1);
    if (hipMalloc(&b->dmem, off) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(DIAQ_ERR_OUT_OF_MEMORY, "batch tables: %zu bytes", off));
    }
    if (ws_elems && hipMalloc(&b->ws, size_t(ws_elems) * sizeof(double2)) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(DIAQ_ERR_OUT_OF_MEMORY, "batch vectors: %lld elements", (long long)ws_elems));
    }
    char* base = static_cast<char*>(b->dmem);
    hipError_t e = hipSuccess;
    auto up = [&](size_t o, const void* src, size_t bytes) {
      if (e == hipSuccess && bytes) e = hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice);
    };
    up(o_circ, circ.data(), circ.size() * sizeof(BCirc));
    up(o_gates, gates.data(), gates.size() * sizeof(BGate));
    up(o_zm, zm.data(), zm.size() * sizeof(uint64_t));
    up(o_coef, coef.data(), coef.size() * sizeof(double));
    up(o_order, narrow.data(), narrow.size() * sizeof(int32_t));
    up(o_wres, wres.data(), wres.size() * sizeof(WideRes));
    up(o_wmeta, wmeta.data(), wmeta.size() * sizeof(WideDot));
    for (size_t x = 0; x < wide.size(); x++) {
      up(o_seg + wide[x].o_fwd, seg_host[2 * x].data(), seg_host[2 * x].size());
      up(o_seg + wide[x].o_rev, seg_host[2 * x + 1].data(), seg_host[2 * x + 1].size());
      wide[x].d_fwd = base + o_seg + wide[x].o_fwd;
      wide[x].d_rev = base + o_seg + wide[x].o_rev;
    }
    for (auto& sp : patches) sp.dst = reinterpret_cast<double*>(base + o_seg + reinterpret_cast<size_t>(sp.dst));
    up(o_patch, patches.data(), patches.size() * sizeof(SegPatch));
    if (e != hipSuccess) return bail(fail(DIAQ_ERR_DEVICE, "batch upload: %s", hipGetErrorString(e)));
    b->args.circ = reinterpret_cast<const BCirc*>(base + o_circ);
    b->args.gates = reinterpret_cast<const BGate*>(base + o_gates);
    b->args.zmask = reinterpret_cast<const uint64_t*>(base + o_zm);
    b->args.coef = reinterpret_cast<const double*>(base + o_coef);
    b->args.order = reinterpret_cast<const int32_t*>(base + o_order);
    b->args.theta = reinterpret_cast<const double*>(base + o_theta);
    b->args.mats = reinterpret_cast<const double*>(base + o_mats);
    b->args.expvals = reinterpret_cast<double*>(base + o_exp);
    b->args.grads = reinterpret_cast<double*>(base + o_grad);
    b->args.queue = reinterpret_cast<int32_t*>(base + o_queue);
    b->args.ws = b->ws;
    b->args.ncirc = int32_t(narrow.size());
    b->d_wres = reinterpret_cast<WideRes*>(base + o_wres);
    b->d_wmeta = reinterpret_cast<WideDot*>(base + o_wmeta);
    b->d_dots = reinterpret_cast<double2*>(base + o_dots);
    b->d_evals = reinterpret_cast<double2*>(base + o_evals);
    b->d_patch = reinterpret_cast<SegPatch*>(base + o_patch);
    b->npatch = int64_t(patches.size());
    // grouped-launch descriptors (they hold the device addresses set above)
    if (!wide.empty()) {
      std::vector<GroupItem> fi, ri;
      std::vector<WideVec> wv;
      int64_t blocks = 0;
      for (size_t x = 0; x < wide.size(); x++) {
        const WideCirc& w = wide[x];
        const int64_t N = int64_t(1) << w.n;
        double2* psi = b->ws + w.s0;
        double2* part = reinterpret_cast<double2*>(base + o_part + w.o_part);
        fi.push_back(GroupItem{&w.fwd, w.d_fwd, w.n, psi, nullptr, nullptr});
        ri.push_back(GroupItem{&w.rev, w.d_rev, w.n, psi, psi + N, part});
        WideVec v;
        std::memset(&v, 0, sizeof(v));
        v.psi = psi;
        v.lam = psi + N;
        v.N = N;
        v.zm = b->args.zmask + w.t0;
        v.coef = b->args.coef + w.t0;
        v.nt = w.nt;
        v.partial = part;
        v.eval = b->d_evals + x;
        v.block0 = blocks;
        blocks += (N + kObsSpan - 1) / kObsSpan;
        wv.push_back(v);
      }
      DIAQ_TRY_BAIL(build_grouped(fi, true, &b->gfwd));
      DIAQ_TRY_BAIL(build_grouped(ri, false, &b->grev));
      const size_t gf = al(b->gfwd.host.size()), gr = al(b->grev.host.size()), gv = al(wv.size() * sizeof(WideVec));
      if (hipMalloc(&b->gmem, gf + gr + gv) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(DIAQ_ERR_OUT_OF_MEMORY, "batch launch tables: %zu bytes", gf + gr + gv));
      }
      char* gb = static_cast<char*>(b->gmem);
      e = hipMemcpy(gb, b->gfwd.host.data(), b->gfwd.host.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(gb + gf, b->grev.host.data(), b->grev.host.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(gb + gf + gr, wv.data(), wv.size() * sizeof(WideVec), hipMemcpyHostToDevice);
      if (e != hipSuccess) return bail(fail(DIAQ_ERR_DEVICE, "batch upload: %s", hipGetErrorString(e)));
      b->gfwd.dev = gb;
      b->grev.dev = gb + gf;
      b->d_wvec = reinterpret_cast<WideVec*>(gb + gf + gr);
      b->wblocks = blocks;
    }
    b->ngates = int64_t(gates.size());
    b->wide = std::move(wide);
    b->pinned_theta = nparams;
    b->pinned_out = ncircuits + nparams;
    if (hipHostMalloc(reinterpret_cast<void**>(&b->pinned), size_t(b->pinned_theta + b->pinned_out + 1) * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(DIAQ_ERR_OUT_OF_MEMORY, "pinned batch buffers"));
    }
    b->lds_bytes = size_t(2) << kLdsMaxQubits;
    b->lds_bytes *= sizeof(double2);
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(batch_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            int(b->lds_bytes)) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(DIAQ_ERR_DEVICE, "cannot reserve %zu bytes of LDS per workgroup", b->lds_bytes));
    }
    b->grid = std::max(1, std::min(ctx->num_cus, b->nnarrow));
    b->graph = (flags & DIAQ_BATCH_GRAPH) != 0;
    *out = b;
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

diaq_status_t diaq_batch_run(diaq_batch_t b, const double* theta, double* expvals, double* grads) {
  if (!b || !expvals || (b->nparams > 0 && !grads)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  if (b->ncirc == 0) return DIAQ_OK;
  const bool use_theta = theta != nullptr;
  if (use_theta) std::memcpy(b->pinned, theta, size_t(b->nparams) * sizeof(double));
  // order after any work the caller queued on the context stream
  DIAQ_HIP(hipStreamSynchronize(b->ctx->stream));
  if (b->graph) {
    if (b->exec && b->have_theta_graph != use_theta) {
      DIAQ_HIP(hipGraphExecDestroy(b->exec));
      DIAQ_HIP(hipGraphDestroy(b->g));
      b->exec = nullptr;
      b->g = nullptr;
    }
    if (!b->exec) {
      DIAQ_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      diaq_status_t st = enqueue(b, use_theta);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(b->stream, &g);
      if (st != DIAQ_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(DIAQ_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
      b->g = g;
      DIAQ_HIP(hipGraphInstantiate(&b->exec, b->g, nullptr, nullptr, 0));
      b->have_theta_graph = use_theta;
    }
    DIAQ_HIP(hipGraphLaunch(b->exec, b->stream));
  } else {
    DIAQ_TRY(enqueue(b, use_theta));
  }
  DIAQ_HIP(hipStreamSynchronize(b->stream));
  const double* out = b->pinned + b->pinned_theta;
  std::memcpy(expvals, out, size_t(b->ncirc) * sizeof(double));
  if (b->nparams) std::memcpy(grads, out + b->ncirc, size_t(b->nparams) * sizeof(double));
  return DIAQ_OK;
}

}  // extern "C"

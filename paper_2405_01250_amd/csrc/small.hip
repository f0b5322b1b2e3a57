// small.hip -- whole circuits on small states in one launch (Alg. 3 in LDS).
//
// Below about 2^13 amplitudes a gate's work is a few microseconds of HBM
// traffic, so the per-gate launches of the in-place path are the cost, not
// the product.  Here one 1024-lane workgroup copies the state into LDS,
// applies a run of gates to it (each Alg. 3 style: the gate's small matrix
// on every coset of its target bits whose controls are 1, in place), with
// a workgroup barrier between gates, and copies the state back.  The gates
// travel in the kernel arguments (a packed list of at most kSmallBlob
// bytes), so a launch needs no table upload; a longer circuit takes one
// launch per run of gates that fits.
#include <cstddef>

#include "internal.hpp"

namespace diaq {

namespace {

constexpr int kSmallThreads = 1024;
constexpr int kSmallBlob = 3840;  // bytes of packed gates per launch

// One packed gate: this header, then the matrix, interleaved complex:
// 2^k entries (the diagonal) when diag, else 4^k entries row-major.
struct SmallGate {
  int32_t k;        // targets, 1..3
  int32_t diag;     // 1: diagonal local matrix
  int32_t t[3];     // target qubits, t[j] = local bit j
  int32_t sorted[3];
  int32_t bytes;    // size of the record (header + matrix)
  int32_t pad;
  uint64_t cmask;   // controls: the gate acts where all are 1
};
static_assert(sizeof(SmallGate) % 16 == 0, "records stay 16-byte aligned");

struct SmallArgs {
  int32_t n;
  int32_t ngates;
  char blob[kSmallBlob];
};
static_assert(offsetof(SmallArgs, blob) == 8, "packed gates start 8 bytes into the arguments");

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

typedef __attribute__((address_space(4))) const char SmallGC;
typedef __attribute__((address_space(4))) const SmallGate SmallGH;
typedef __attribute__((address_space(4))) const double SmallGD;

// The 2^K amplitudes of coset c (controls checked by the caller) times the
// gate's dense matrix, in place in LDS.
template <int K>
__device__ __forceinline__ void small_coset(double2* st, int64_t base, const int64_t (&off)[8], SmallGD* m) {
  constexpr int D = 1 << K;
  double xr[D], xi[D];
#pragma unroll
  for (int r = 0; r < D; r++) {
    const double2 t = st[base + off[r]];
    xr[r] = t.x;
    xi[r] = t.y;
  }
#pragma unroll
  for (int r = 0; r < D; r++) {
    double yr = 0, yi = 0;
#pragma unroll
    for (int c = 0; c < D; c++) {
      const double mr = m[2 * (r * D + c)], mi = m[2 * (r * D + c) + 1];
      yr = fma(mr, xr[c], fma(-mi, xi[c], yr));
      yi = fma(mr, xi[c], fma(mi, xr[c], yi));
    }
    st[base + off[r]] = double2{yr, yi};
  }
}

template <typename R>
__global__ __launch_bounds__(kSmallThreads) void small_circuit_kernel(SmallArgs a, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  extern __shared__ double2 st[];
  const int64_t N = int64_t(1) << a.n;
  for (int64_t i = threadIdx.x; i < N; i += kSmallThreads) {
    const V t = v[i];
    st[i] = double2{double(t.x), double(t.y)};
  }
  __syncthreads();
  // the packed gates are read where the kernel arguments live: `a` is the
  // first argument, at offset 0 of the kernel-argument segment (taking the
  // address of the by-value parameter itself would copy it to scratch
  // memory, whose addresses are not constant-space addresses)
  SmallGC* p = (SmallGC*)(__builtin_amdgcn_kernarg_segment_ptr()) + offsetof(SmallArgs, blob);
  for (int g = 0; g < a.ngates; g++) {
    SmallGH* h = (SmallGH*)(p);
    SmallGD* m = (SmallGD*)(p + sizeof(SmallGate));
    const int k = h->k;
    const uint64_t cmask = h->cmask;
    if (h->diag) {
      // element-wise: row r of the local diagonal from the target bits
      for (int64_t i = threadIdx.x; i < N; i += kSmallThreads) {
        if ((uint64_t(i) & cmask) != cmask) continue;
        int r = 0;
        for (int j = 0; j < k; j++) r |= int((i >> h->t[j]) & 1) << j;
        const double fr = m[2 * r], fi = m[2 * r + 1];
        const double2 x = st[i];
        st[i] = double2{fma(x.x, fr, -x.y * fi), fma(x.x, fi, x.y * fr)};
      }
    } else {
      int64_t off[8];
#pragma unroll
      for (int r = 0; r < 8; r++) {
        int64_t o = 0;
        for (int j = 0; j < k; j++)
          if ((r >> j) & 1) o |= int64_t(1) << h->t[j];
        off[r] = o;
      }
      const int64_t C = N >> k;
      for (int64_t c = threadIdx.x; c < C; c += kSmallThreads) {
        int64_t base = c;
        for (int j = 0; j < k; j++) {
          const int q = h->sorted[j];
          base = (base & ((int64_t(1) << q) - 1)) | ((base >> q) << (q + 1));
        }
        if ((uint64_t(base) & cmask) != cmask) continue;
        if (k == 1) small_coset<1>(st, base, off, m);
        else if (k == 2) small_coset<2>(st, base, off, m);
        else small_coset<3>(st, base, off, m);
      }
    }
    p += h->bytes;
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < N; i += kSmallThreads) {
    const double2 t = st[i];
    v[i] = V{R(t.x), R(t.y)};
  }
}

bool diagonal_local(const LocalGate& lg) {
  for (int r = 0; r < (1 << lg.k); r++)
    for (int c = 0; c < (1 << lg.k); c++)
      if (r != c && lg.structural[r][c]) return false;
  return true;
}

// Appends lg's record to blob; false (blob unchanged) if it does not fit.
bool pack_gate(const LocalGate& lg, std::vector<char>* blob) {
  const int D = 1 << lg.k;
  const bool diag = diagonal_local(lg);
  const size_t mbytes = size_t(diag ? D : D * D) * 16;
  const size_t bytes = sizeof(SmallGate) + mbytes;
  if (blob->size() + bytes > size_t(kSmallBlob)) return false;
  SmallGate h;
  std::memset(&h, 0, sizeof(h));
  h.k = lg.k;
  h.diag = diag ? 1 : 0;
  int s[3] = {0, 0, 0};
  for (int j = 0; j < lg.k; j++) h.t[j] = s[j] = lg.targets[j];
  std::sort(s, s + lg.k);
  for (int j = 0; j < lg.k; j++) h.sorted[j] = s[j];
  h.bytes = int32_t(bytes);
  h.cmask = lg.cmask;
  const size_t at = blob->size();
  blob->resize(at + bytes);
  std::memcpy(blob->data() + at, &h, sizeof(h));
  double* m = reinterpret_cast<double*>(blob->data() + at + sizeof(h));
  if (diag) {
    for (int r = 0; r < D; r++) {
      m[2 * r] = lg.m[r][r][0];
      m[2 * r + 1] = lg.m[r][r][1];
    }
  } else {
    for (int r = 0; r < D; r++)
      for (int c = 0; c < D; c++) {
        m[2 * (r * D + c)] = lg.m[r][c][0];
        m[2 * (r * D + c) + 1] = lg.m[r][c][1];
      }
  }
  return true;
}

}  // namespace

int small_circuit_qubits(const diaq_ctx* ctx, diaq_dtype_t dt) {
  const int knob = ctx->tuning.kron_small_qubits;
  if (knob < 0) return 0;
  // the state is held as complex128 in LDS whatever its type
  int fit = 0;
  while (fit < 14 && (size_t(16) << (fit + 1)) <= size_t(ctx->lds_bytes)) fit++;
  (void)dt;
  return knob == 0 ? fit : std::min(knob, fit);
}

diaq_status_t run_small(diaq_ctx* ctx, const std::vector<LocalGate>& lg, int n, diaq_dtype_t dt, void* state) {
  if (n > small_circuit_qubits(ctx, dt)) return fail(DIAQ_ERR_UNSUPPORTED, "state of %d qubits does not fit LDS", n);
  const int64_t N = int64_t(1) << n;
  const size_t lds = size_t(N) * sizeof(double2);
  static bool raised[2] = {false, false};  // LDS limit lifted once per kernel
  const int ti = dt == DIAQ_C128 ? 0 : 1;
  if (lds > 65536 && !raised[ti]) {
    const void* fn = dt == DIAQ_C128 ? reinterpret_cast<const void*>(&small_circuit_kernel<double>)
                                     : reinterpret_cast<const void*>(&small_circuit_kernel<float>);
    DIAQ_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, ctx->lds_bytes));
    raised[ti] = true;
  }
  const double bytes = 2.0 * double(elem_bytes(dt)) * double(N);
  size_t g = 0;
  while (g < lg.size()) {
    SmallArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    std::vector<char> blob;
    blob.reserve(kSmallBlob);
    while (g < lg.size() && pack_gate(lg[g], &blob)) {
      a.ngates++;
      g++;
    }
    if (a.ngates == 0) return fail(DIAQ_ERR_DEVICE, "gate %zu does not fit a launch", g);
    std::memcpy(a.blob, blob.data(), blob.size());
    const size_t e0 = prof_mark(ctx);
    if (dt == DIAQ_C128)
      hipLaunchKernelGGL(small_circuit_kernel<double>, dim3(1), dim3(kSmallThreads), lds, ctx->stream, a,
                         static_cast<double2*>(state));
    else
      hipLaunchKernelGGL(small_circuit_kernel<float>, dim3(1), dim3(kSmallThreads), lds, ctx->stream, a,
                         static_cast<float2*>(state));
    DIAQ_HIP(hipGetLastError());
    prof_interval(ctx, e0, prof_mark(ctx), 1, bytes);
  }
  return DIAQ_OK;
}

}  // namespace diaq

// api.cpp -- the C entry points of libdiaq_hip: context, DiaQ matrix
// objects, gate expansion, products and expectation values.
#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <new>
#include <set>

#include "internal.hpp"

namespace diaq {

namespace {
thread_local char g_err[512] = "";
}

diaq_status_t fail(diaq_status_t st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_err[0] = 0; }

diaq_status_t ensure(diaq_ctx* ctx, Workspace* w, size_t bytes) {
  if (ctx->capture) {
    // nothing may be allocated or freed while a graph is being recorded
    if (ctx->capture->sizing) {
      w->want = std::max(w->want, bytes);
      return DIAQ_OK;
    }
    if (w->bytes < bytes)
      return fail(DIAQ_ERR_DEVICE, "graph workspace of %zu bytes, %zu needed", w->bytes, bytes);
    return DIAQ_OK;
  }
  if (w->bytes >= bytes) return DIAQ_OK;
  if (w->ptr) {
    // work queued on the stream may still use the old buffer
    DIAQ_HIP(hipStreamSynchronize(ctx->stream));
    DIAQ_HIP(hipFree(w->ptr));
    w->ptr = nullptr;
    w->bytes = 0;
  }
  const size_t want = std::max<size_t>(bytes, 4096);
  hipError_t e = hipMalloc(&w->ptr, want);
  if (e != hipSuccess) {
    w->ptr = nullptr;
    (void)hipGetLastError();
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "hipMalloc(%zu bytes) failed: %s", want, hipGetErrorString(e));
  }
  w->bytes = want;
  return DIAQ_OK;
}

diaq_status_t upload(diaq_ctx* ctx, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return DIAQ_OK;
  if (Capture* c = ctx->capture) {
    const size_t span = (bytes + 255) & ~size_t(255);
    if (c->sizing) {
      c->host_used += span;
      return DIAQ_OK;
    }
    if (c->host_used + span > c->host_bytes)
      return fail(DIAQ_ERR_DEVICE, "graph staging of %zu bytes overrun", c->host_bytes);
    char* h = c->host + c->host_used;
    std::memcpy(h, src, bytes);
    c->host_used += span;
    DIAQ_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, ctx->stream));
    return DIAQ_OK;
  }
  // earlier work on the stream may still read the previous contents
  DIAQ_HIP(hipStreamSynchronize(ctx->stream));
  DIAQ_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  return DIAQ_OK;
}

diaq_status_t ensure_pinned(diaq_ctx* ctx, size_t bytes) {
  if (ctx->pinned_bytes >= bytes) return DIAQ_OK;
  if (ctx->pinned) {
    DIAQ_HIP(hipStreamSynchronize(ctx->stream));
    DIAQ_HIP(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
  }
  const size_t want = std::max<size_t>(bytes, 4096);
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "hipHostMalloc(%zu) failed: %s", want, hipGetErrorString(e));
  }
  ctx->pinned = static_cast<double*>(p);
  ctx->pinned_bytes = want;
  return DIAQ_OK;
}

diaq_status_t new_dia(diaq_ctx* ctx, int n, diaq_dtype_t dt, const std::vector<int64_t>& offs, void* values,
                      bool zero_fill, diaq_dia** out) {
  diaq_dia* m = new (std::nothrow) diaq_dia();
  if (!m) return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  m->nqubits = n;
  m->ndiag = int32_t(offs.size());
  m->dtype = dt;
  m->offsets = offs;
  m->starts = packing_starts(offs, n);
  m->qubit_mask = mask_from_offsets(offs);
  m->device = ctx->device;
  const size_t bytes = size_t(m->starts.back()) * elem_bytes(dt);
  if (values) {
    m->values = values;
    m->owns_values = false;
  } else if (bytes) {
    hipError_t e = hipMalloc(&m->values, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      delete m;
      return fail(DIAQ_ERR_OUT_OF_MEMORY, "hipMalloc(%zu bytes) for diagonals failed", bytes);
    }
    m->owns_values = true;
    if (zero_fill) {
      e = hipMemsetAsync(m->values, 0, bytes, ctx->stream);
      if (e != hipSuccess) {
        (void)hipFree(m->values);
        delete m;
        return fail(DIAQ_ERR_DEVICE, "hipMemsetAsync failed: %s", hipGetErrorString(e));
      }
    }
  }
  if (m->ndiag > kMaxArgDiags) {
    // device copy of offsets and starts for kernels that cannot take them by value
    const size_t mb = (2 * size_t(m->ndiag) + 1) * sizeof(int64_t);
    hipError_t e = hipMalloc(&m->dmeta, mb);
    if (e == hipSuccess)
      e = hipMemcpy(m->dmeta, m->offsets.data(), m->ndiag * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(m->dmeta + m->ndiag, m->starts.data(), (m->ndiag + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (m->dmeta) (void)hipFree(m->dmeta);
      if (m->owns_values) (void)hipFree(m->values);
      delete m;
      return fail(DIAQ_ERR_OUT_OF_MEMORY, "device offset table: %s", hipGetErrorString(e));
    }
  }
  *out = m;
  return DIAQ_OK;
}

size_t prof_mark(diaq_ctx* ctx) {
  if (!ctx->profiling) return SIZE_MAX;
  if (ctx->events_used == ctx->events.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return SIZE_MAX;
    }
    ctx->events.push_back(e);
  }
  const size_t i = ctx->events_used;
  if (hipEventRecord(ctx->events[i], ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    return SIZE_MAX;
  }
  ctx->events_used++;
  return i;
}

void prof_interval(diaq_ctx* ctx, size_t ev0, size_t ev1, int kind, double bytes) {
  if (!ctx->profiling || ev0 == SIZE_MAX || ev1 == SIZE_MAX) return;
  ctx->intervals.push_back({ev0, ev1, kind, bytes});
}

SpmvOp op_of(const diaq_dia* A, bool transpose, bool conjugate) {
  SpmvOp op;
  op.n = A->nqubits;
  op.dtype = A->dtype;
  op.nd = A->ndiag;
  op.host_off = A->offsets.data();
  op.host_start = A->starts.data();
  op.dmeta = A->dmeta;
  op.values = A->values;
  op.transpose = transpose;
  op.conjugate = conjugate;
  op.qubit_mask = A->qubit_mask;
  op.skip_zero = A->layout_zeros;
  return op;
}

}  // namespace diaq

using namespace diaq;

#define DIAQ_GUARD_BEGIN try {
#define DIAQ_GUARD_END                                                   \
  }                                                                      \
  catch (const std::bad_alloc&) {                                        \
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");       \
  }                                                                      \
  catch (...) {                                                          \
    return fail(DIAQ_ERR_DEVICE, "unexpected C++ exception");            \
  }

extern "C" {

const char* diaq_last_error(void) { return g_err; }

const char* diaq_status_string(diaq_status_t s) {
  switch (s) {
    case DIAQ_OK: return "ok";
    case DIAQ_ERR_INVALID_ARGUMENT: return "invalid argument";
    case DIAQ_ERR_NOT_MULTIPLYABLE: return "not multiplyable";
    case DIAQ_ERR_OUT_OF_MEMORY: return "out of memory";
    case DIAQ_ERR_DEVICE: return "device error";
    case DIAQ_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

diaq_status_t diaq_create(int32_t device, void* hip_stream, diaq_ctx_t* out) {
  DIAQ_GUARD_BEGIN
  if (!out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "out is NULL");
  int count = 0;
  DIAQ_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "device %d not in [0, %d)", device, count);
  DIAQ_HIP(hipSetDevice(device));
  // the device address of the static scratch array, once per device
  DIAQ_TRY(init_static_scratch(device));
  diaq_ctx* c = new diaq_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->num_cus = cus;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    c->lds_bytes = lds;
  *out = c;
  clear_error();
  return DIAQ_OK;
  DIAQ_GUARD_END
}

diaq_status_t diaq_set_stream(diaq_ctx_t ctx, void* hip_stream) {
  if (!ctx) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return DIAQ_OK;
}

diaq_status_t diaq_synchronize(diaq_ctx_t ctx) {
  if (!ctx) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx is NULL");
  DIAQ_HIP(hipStreamSynchronize(ctx->stream));
  return DIAQ_OK;
}

static diaq_status_t check_tuning(const diaq_tuning_t* t) {
  if (t->spmv_rows != 0 && t->spmv_rows != 1 && t->spmv_rows != 2 && t->spmv_rows != 4)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "spmv_rows must be 0, 1, 2 or 4");
  if (t->spmv_group_bits < -1 || t->spmv_group_bits > 3)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "spmv_group_bits must be in [-1, 3]");
  if (t->spmv_chunk != 0 && t->spmv_chunk != 1 && t->spmv_chunk != 3)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "spmv_chunk must be 0, 1 or 3");
  if (t->diag_pad < -1 || t->diag_pad > (1 << 24))
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "diag_pad must be in [-1, 2^24]");
  if (t->spmv_group_min_qubit < 0 || t->spmv_group_min_qubit > 63)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "spmv_group_min_qubit must be in [0, 63]");
  if (t->spmv_xcd_runs != 0 && t->spmv_xcd_runs != -1)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "spmv_xcd_runs must be 0 or -1");
  if (t->kron_stage_qubit < -1 || t->kron_stage_qubit > 6)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "kron_stage_qubit must be in [-1, 6]");
  if (t->kron_split < 0 || t->kron_split > 7) return fail(DIAQ_ERR_INVALID_ARGUMENT, "kron_split must be in [0, 7]");
  if (t->kron_nontemporal < -1 || t->kron_nontemporal > 1)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "kron_nontemporal must be -1, 0 or 1");
  if (t->kron_small_qubits < -1 || t->kron_small_qubits > 14)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "kron_small_qubits must be in [-1, 14]");
  if (t->kron_order < 0 || t->kron_order > 3) return fail(DIAQ_ERR_INVALID_ARGUMENT, "kron_order must be 0..3");
  if (t->spmv_order < 0 || t->spmv_order > 2) return fail(DIAQ_ERR_INVALID_ARGUMENT, "spmv_order must be 0, 1 or 2");
  if (t->spmv_pack < -1 || t->spmv_pack > 0) return fail(DIAQ_ERR_INVALID_ARGUMENT, "spmv_pack must be 0 or -1");
  return DIAQ_OK;
}

diaq_status_t diaq_set_tuning(diaq_ctx_t ctx, const diaq_tuning_t* t) {
  if (!ctx || !t) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  DIAQ_TRY(check_tuning(t));
  ctx->tuning = *t;
  return DIAQ_OK;
}

diaq_status_t diaq_spmv_shape(const diaq_gate_t* gate, int32_t nqubits, diaq_dtype_t dtype, const diaq_tuning_t* t,
                              diaq_spmv_shape_t* out) {
  DIAQ_GUARD_BEGIN
  if (!gate || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  if (dtype != DIAQ_C64 && dtype != DIAQ_C128) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad dtype");
  diaq_tuning_t tt{};
  if (t) {
    DIAQ_TRY(check_tuning(t));
    tt = *t;
  }
  LocalGate lg;
  DIAQ_TRY(local_gate(gate, nqubits, &lg));
  const std::vector<int64_t> offs = gate_offsets(lg);
  if (offs.empty()) return fail(DIAQ_ERR_INVALID_ARGUMENT, "the gate's matrix is zero");
  const std::vector<int64_t> st = packing_starts(offs, nqubits);
  SpmvOp op;
  op.n = nqubits;
  op.dtype = dtype;
  op.nd = int(offs.size());
  op.host_off = offs.data();
  op.host_start = st.data();
  op.qubit_mask = lg.tmask;
  op.skip_zero = true;
  return spmv_shape(op, tt, out);
  DIAQ_GUARD_END
}

diaq_status_t diaq_get_tuning(diaq_ctx_t ctx, diaq_tuning_t* t) {
  if (!ctx || !t) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  *t = ctx->tuning;
  return DIAQ_OK;
}

diaq_status_t diaq_profile_start(diaq_ctx_t ctx) {
  if (!ctx) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx is NULL");
  ctx->profiling = true;
  ctx->events_used = 0;
  ctx->intervals.clear();
  return DIAQ_OK;
}

diaq_status_t diaq_profile_stop(diaq_ctx_t ctx, diaq_profile_t* out) {
  if (!ctx || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  DIAQ_HIP(hipStreamSynchronize(ctx->stream));
  for (const auto& iv : ctx->intervals) {
    float ms = 0;
    DIAQ_HIP(hipEventElapsedTime(&ms, ctx->events[iv.ev0], ctx->events[iv.ev1]));
    if (iv.kind == 0) {
      out->expand_launches++;
      out->expand_ms += ms;
      out->expand_bytes += iv.bytes;
    } else {
      out->spmv_launches++;
      out->spmv_ms += ms;
      out->spmv_bytes += iv.bytes;
    }
  }
  ctx->profiling = false;
  ctx->events_used = 0;
  ctx->intervals.clear();
  return DIAQ_OK;
}

diaq_status_t diaq_destroy(diaq_ctx_t ctx) {
  if (!ctx) return DIAQ_OK;
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  for (Workspace* w : {&ctx->diag, &ctx->red, &ctx->aux})
    if (w->ptr) (void)hipFree(w->ptr);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return DIAQ_OK;
}

diaq_status_t diaq_dia_create(diaq_ctx_t ctx, int32_t nqubits, diaq_dtype_t dtype, int32_t ndiag,
                              const int64_t* offsets, void* values, diaq_dia_t* out) {
  DIAQ_GUARD_BEGIN
  if (!ctx || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx/out is NULL");
  if (nqubits < 1 || nqubits > 34) return fail(DIAQ_ERR_INVALID_ARGUMENT, "nqubits %d out of range", nqubits);
  if (dtype != DIAQ_C64 && dtype != DIAQ_C128) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad dtype %d", int(dtype));
  if (ndiag < 0 || (ndiag > 0 && !offsets)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad diagonal list");
  const int64_t N = int64_t(1) << nqubits;
  std::vector<int64_t> offs(offsets, offsets + ndiag);
  for (int k = 0; k < ndiag; k++) {
    if (offs[k] <= -N || offs[k] >= N)
      return fail(DIAQ_ERR_INVALID_ARGUMENT, "diagonal index %lld outside (-N, N)", (long long)offs[k]);
    if (k && offs[k] <= offs[k - 1]) return fail(DIAQ_ERR_INVALID_ARGUMENT, "diagonal indices not strictly ascending");
  }
  if (values && (reinterpret_cast<uintptr_t>(values) & 15))
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "values pointer not 16-byte aligned");
  diaq_dia* m = nullptr;
  DIAQ_TRY(new_dia(ctx, nqubits, dtype, offs, values, true, &m));
  *out = m;
  return DIAQ_OK;
  DIAQ_GUARD_END
}

diaq_status_t diaq_dia_info(diaq_dia_t A, int32_t* nqubits, int32_t* ndiag, int32_t* dtype, int64_t* nvalues,
                            void** values) {
  if (!A) return fail(DIAQ_ERR_INVALID_ARGUMENT, "matrix is NULL");
  if (nqubits) *nqubits = A->nqubits;
  if (ndiag) *ndiag = A->ndiag;
  if (dtype) *dtype = A->dtype;
  if (nvalues) *nvalues = A->starts.back();
  if (values) *values = A->values;
  return DIAQ_OK;
}

diaq_status_t diaq_dia_offsets(diaq_dia_t A, int64_t* offsets, int64_t* starts) {
  if (!A) return fail(DIAQ_ERR_INVALID_ARGUMENT, "matrix is NULL");
  // report the matrix as applied: a transposed view lists negated indices
  // in ascending order, each with the start of the storage it reads
  const int nd = A->ndiag;
  for (int k = 0; k < nd; k++) {
    const int kk = A->transposed ? nd - 1 - k : k;
    if (offsets) offsets[k] = A->transposed ? -A->offsets[kk] : A->offsets[kk];
    if (starts) starts[k] = A->starts[kk];
  }
  if (starts) starts[nd] = A->starts[nd];
  return DIAQ_OK;
}

diaq_status_t diaq_dia_transpose(diaq_dia_t A, int32_t conjugate, diaq_dia_t* out) {
  DIAQ_GUARD_BEGIN
  if (!A || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "matrix/out is NULL");
  diaq_dia* m = new diaq_dia(*A);
  m->owns_values = false;
  m->dmeta = nullptr;
  if (A->dmeta) {
    const size_t mb = (2 * size_t(m->ndiag) + 1) * sizeof(int64_t);
    DIAQ_HIP(hipMalloc(&m->dmeta, mb));
    DIAQ_HIP(hipMemcpy(m->dmeta, A->dmeta, mb, hipMemcpyDeviceToDevice));
  }
  m->transposed = !A->transposed;
  if (conjugate) m->conjugated = !A->conjugated;
  *out = m;
  return DIAQ_OK;
  DIAQ_GUARD_END
}

diaq_status_t diaq_dia_copy_values(diaq_ctx_t ctx, diaq_dia_t A, void* dst, int32_t dst_on_host) {
  if (!ctx || !A || !dst) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  const size_t bytes = size_t(A->starts.back()) * elem_bytes(A->dtype);
  if (!bytes) return DIAQ_OK;
  DIAQ_HIP(hipMemcpyAsync(dst, A->values, bytes, dst_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                          ctx->stream));
  DIAQ_HIP(hipStreamSynchronize(ctx->stream));
  return DIAQ_OK;
}

diaq_status_t diaq_dia_free(diaq_dia_t A) {
  if (!A) return DIAQ_OK;
  if (A->owns_values && A->values) (void)hipFree(A->values);
  if (A->dmeta) (void)hipFree(A->dmeta);
  delete A;
  return DIAQ_OK;
}

diaq_status_t diaq_from_gate_query(const diaq_gate_t* gate, int32_t nqubits, int32_t* ndiag, int64_t* offsets,
                                   int64_t* nvalues) {
  DIAQ_GUARD_BEGIN
  LocalGate lg;
  DIAQ_TRY(local_gate(gate, nqubits, &lg));
  const std::vector<int64_t> offs = gate_offsets(lg);
  if (ndiag) *ndiag = int32_t(offs.size());
  if (offsets) std::copy(offs.begin(), offs.end(), offsets);
  if (nvalues) *nvalues = packing_starts(offs, nqubits).back();
  return DIAQ_OK;
  DIAQ_GUARD_END
}

diaq_status_t diaq_from_gate(diaq_ctx_t ctx, const diaq_gate_t* gate, int32_t nqubits, diaq_dtype_t dtype,
                             diaq_dia_t* out) {
  DIAQ_GUARD_BEGIN
  if (!ctx || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx/out is NULL");
  if (dtype != DIAQ_C64 && dtype != DIAQ_C128) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad dtype");
  LocalGate lg;
  DIAQ_TRY(local_gate(gate, nqubits, &lg));
  const std::vector<int64_t> offs = gate_offsets(lg);
  diaq_dia* m = nullptr;
  DIAQ_TRY(new_dia(ctx, nqubits, dtype, offs, nullptr, false, &m));
  m->qubit_mask = lg.tmask;
  m->layout_zeros = true;
  diaq_status_t st = launch_expand(ctx, lg, nqubits, dtype, m->offsets, m->starts, m->values);
  if (st != DIAQ_OK) {
    diaq_dia_free(m);
    return st;
  }
  *out = m;
  return DIAQ_OK;
  DIAQ_GUARD_END
}

diaq_status_t diaq_from_pauli_sum(diaq_ctx_t ctx, int32_t nqubits, diaq_dtype_t dtype, int32_t nterms,
                                  const uint64_t* xmask, const uint64_t* zmask, const double* coef,
                                  diaq_dia_t* out) {
  DIAQ_GUARD_BEGIN
  if (!ctx || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx/out is NULL");
  if (nqubits < 1 || nqubits > 34) return fail(DIAQ_ERR_INVALID_ARGUMENT, "nqubits out of range");
  if (nterms < 0 || (nterms > 0 && (!xmask || !zmask || !coef)))
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad term arrays");
  const uint64_t full = (nqubits == 64) ? ~0ull : ((1ull << nqubits) - 1);
  std::set<int64_t> offset_set;
  uint64_t qmask = 0;
  for (int t = 0; t < nterms; t++) {
    if ((xmask[t] | zmask[t]) & ~full) return fail(DIAQ_ERR_INVALID_ARGUMENT, "term %d acts outside the register", t);
    // diagonal (i xor x) - i over all i: each flipped bit contributes +-2^q
    int bits[64], nb = 0;
    for (int q = 0; q < nqubits; q++)
      if ((xmask[t] >> q) & 1) bits[nb++] = q;
    if (nb > 16) return fail(DIAQ_ERR_UNSUPPORTED, "term %d flips %d qubits", t, nb);
    for (int s = 0; s < (1 << nb); s++) {
      int64_t d = 0;
      for (int b = 0; b < nb; b++) d += ((s >> b) & 1) ? -(int64_t(1) << bits[b]) : (int64_t(1) << bits[b]);
      offset_set.insert(d);
    }
    qmask |= xmask[t];
  }
  std::vector<int64_t> offs(offset_set.begin(), offset_set.end());
  diaq_dia* m = nullptr;
  DIAQ_TRY(new_dia(ctx, nqubits, dtype, offs, nullptr, false, &m));
  m->qubit_mask = qmask;
  m->layout_zeros = true;
  diaq_status_t st = launch_pauli_dia(ctx, nqubits, dtype, m->offsets, m->starts, xmask, zmask, coef, nterms,
                                      m->values);
  if (st != DIAQ_OK) {
    diaq_dia_free(m);
    return st;
  }
  *out = m;
  return DIAQ_OK;
  DIAQ_GUARD_END
}

diaq_status_t diaq_spmv(diaq_ctx_t ctx, diaq_dia_t A, const void* x, void* y, uint32_t flags) {
  DIAQ_GUARD_BEGIN
  if (!ctx || !A || !x || !y) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  if (flags & ~DIAQ_ADJOINT) return fail(DIAQ_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", flags);
  const size_t bytes = (size_t(1) << A->nqubits) * elem_bytes(A->dtype);
  const char* xb = static_cast<const char*>(x);
  const char* yb = static_cast<const char*>(y);
  if (x != y && xb < yb + bytes && yb < xb + bytes)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "x and y overlap");
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "x/y not 16-byte aligned");
  const bool tr = ((flags & DIAQ_TRANSPOSE) != 0) != A->transposed;
  const bool cj = ((flags & DIAQ_CONJUGATE) != 0) != A->conjugated;
  return launch_spmv(ctx, op_of(A, tr, cj), x, y);
  DIAQ_GUARD_END
}

diaq_status_t diaq_fuse(diaq_ctx_t ctx, diaq_dia_t first, diaq_dia_t second, double drop_tol, diaq_dia_t* out) {
  DIAQ_GUARD_BEGIN
  if (!ctx || !first || !second || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  if (first->nqubits != second->nqubits)
    return fail(DIAQ_ERR_NOT_MULTIPLYABLE, "not multiplyable: 2^%d vs 2^%d", first->nqubits, second->nqubits);
  if (first->dtype != second->dtype) return fail(DIAQ_ERR_NOT_MULTIPLYABLE, "not multiplyable: dtypes differ");
  if (!(drop_tol >= 0)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "drop_tol must be >= 0");
  diaq_dia* m = nullptr;
  DIAQ_TRY(fuse_dia(ctx, first, second, drop_tol, &m));
  *out = m;
  return DIAQ_OK;
  DIAQ_GUARD_END
}

diaq_status_t diaq_expect(diaq_ctx_t ctx, diaq_dia_t H, const void* psi, const void* phi, double* out) {
  DIAQ_GUARD_BEGIN
  if (!ctx || !H || !psi || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  DIAQ_TRY(ensure(ctx, &ctx->aux, 256));
  double* dres = static_cast<double*>(ctx->aux.ptr);
  DIAQ_TRY(launch_expect(ctx, op_of(H, H->transposed, H->conjugated), psi, phi ? phi : psi, dres));
  DIAQ_TRY(ensure_pinned(ctx, 2 * sizeof(double)));
  DIAQ_HIP(hipMemcpyAsync(ctx->pinned, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  DIAQ_HIP(hipStreamSynchronize(ctx->stream));
  out[0] = ctx->pinned[0];
  out[1] = ctx->pinned[1];
  return DIAQ_OK;
  DIAQ_GUARD_END
}

diaq_status_t diaq_expect_noalloc(diaq_ctx_t ctx, diaq_dia_t H, const void* psi, const void* phi, double* dres) {
  DIAQ_GUARD_BEGIN
  if (!ctx || !H || !psi || !dres) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(psi) | reinterpret_cast<uintptr_t>(phi) | reinterpret_cast<uintptr_t>(dres)) & 15)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "psi, phi and dres must be 16-byte aligned");
  return launch_expect_static(ctx, op_of(H, H->transposed, H->conjugated), psi, phi ? phi : psi, dres);
  DIAQ_GUARD_END
}

}  // extern "C"

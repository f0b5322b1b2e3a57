// circuit.cpp -- circuit-level drivers: plain per-gate state evolution and
// the adjoint (reverse-sweep) gradient.
//
// State evolution (Sec. II-A, Sec. VI): each gate's time-step unitary is
// expanded into the context's diagonal workspace and applied by the DiaQ
// SpMV, ping-ponging between the caller's state and scratch vectors.  All
// work is queued on one stream; nothing returns to the host until the
// caller reads the state.
#include <algorithm>
#include <cstring>

#include <map>

#include "internal.hpp"

namespace diaq {

namespace {

struct Prepared {
  std::vector<LocalGate> lg;
  std::vector<std::vector<int64_t>> offs;
  int64_t max_values = 0;
};

diaq_status_t prepare_gates(const diaq_gate_t* gates, int64_t ngates, int n, Prepared* p) {
  p->lg.resize(size_t(ngates));
  p->offs.resize(size_t(ngates));
  for (int64_t g = 0; g < ngates; g++) {
    diaq_status_t st = local_gate(&gates[g], n, &p->lg[g]);
    if (st != DIAQ_OK) return fail(st, "gate %lld: %s", (long long)g, diaq_last_error());
    p->offs[g] = gate_offsets(p->lg[g]);
    p->max_values = std::max<int64_t>(p->max_values, packing_starts(p->offs[g], n).back());
  }
  return DIAQ_OK;
}

// Expand gate g into the workspace and apply it (or its adjoint) from *x
// into *y; swaps the pointers unless the gate ran in place.
// Packing starts in the circuit workspace: the compact diagonals one after
// another, each starting on a kStartAlign-byte boundary (a gate on qubit q
// < 4 would otherwise start its later diagonals 16 2^q bytes off one, and
// every store and load of those streams would straddle cache lines),
// optionally separated by ctx->tuning.diag_pad more elements so that the
// streams of one product do not sit at power-of-two distances.
constexpr int64_t kStartAlign = 256;
std::vector<int64_t> workspace_starts(const diaq_ctx* ctx, const std::vector<int64_t>& offs, int n,
                                      diaq_dtype_t dt) {
  const std::vector<int64_t> packed = packing_starts(offs, n);
  const int64_t pad = ctx->tuning.diag_pad > 0 ? ctx->tuning.diag_pad : 0;
  const int64_t a = kStartAlign / int64_t(elem_bytes(dt));
  std::vector<int64_t> st(packed.size());
  int64_t cur = 0;
  for (size_t k = 0; k + 1 < packed.size(); k++) {
    st[k] = (cur + a - 1) / a * a;
    cur = st[k] + (packed[k + 1] - packed[k]) + pad;
  }
  st.back() = cur;
  return st;
}
// Workspace elements beyond the packed values that alignment and padding
// may add to an operation of at most kMaxArgDiags diagonals.
int64_t workspace_slack(const diaq_ctx* ctx, diaq_dtype_t dt) {
  const int64_t pad = ctx->tuning.diag_pad > 0 ? ctx->tuning.diag_pad : 0;
  return int64_t(kMaxArgDiags + 1) * (pad + kStartAlign / int64_t(elem_bytes(dt)));
}

diaq_status_t step(diaq_ctx* ctx, const LocalGate& lg, const std::vector<int64_t>& offs, int n, diaq_dtype_t dt,
                   bool adjoint, void** x, void** y, const char* tabs = nullptr, int nt = 0) {
  const std::vector<int64_t> st = workspace_starts(ctx, offs, n, dt);
  const double s = double(elem_bytes(dt));
  const double E = double(packing_starts(offs, n).back()), N = double(int64_t(1) << n);
  const size_t e0 = prof_mark(ctx);
  DIAQ_TRY(launch_expand(ctx, lg, n, dt, offs, st, ctx->diag.ptr, tabs, nt));
  const size_t e1 = prof_mark(ctx);
  prof_interval(ctx, e0, e1, 0, s * E);
  struct Close {
    diaq_ctx* c;
    size_t e1;
    double bytes;
    ~Close() { prof_interval(c, e1, prof_mark(c), 1, bytes); }
  } close_spmv{ctx, e1, s * (E + 2 * N)};
  SpmvOp op;
  op.n = n;
  op.dtype = dt;
  op.nd = int(offs.size());
  op.host_off = offs.data();
  op.host_start = st.data();
  op.values = ctx->diag.ptr;
  op.transpose = adjoint;
  op.conjugate = adjoint;
  op.qubit_mask = lg.tmask;
  op.skip_zero = true;
  if (offs.empty()) {
    // a gate whose matrix is all zero: y = 0 (a fill kernel, no memset node
    // in a recorded graph)
    DIAQ_TRY(launch_zero(ctx->stream, *y, size_t(int64_t(1) << n) * elem_bytes(dt)));
    std::swap(*x, *y);
    return DIAQ_OK;
  }
  if (offs.size() == 1 && offs[0] == 0) return launch_spmv(ctx, op, *x, *x);
  DIAQ_TRY(launch_spmv(ctx, op, *x, *y));
  std::swap(*x, *y);
  return DIAQ_OK;
}

diaq_status_t check_vectors(int n, diaq_dtype_t dt, const void* a, const void* b) {
  if (dt != DIAQ_C64 && dt != DIAQ_C128) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad dtype");
  if (n < 1 || n > 34) return fail(DIAQ_ERR_INVALID_ARGUMENT, "nqubits %d out of range", n);
  if (!a || !b) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL vector");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "vector not 16-byte aligned");
  const size_t bytes = (size_t(1) << n) * elem_bytes(dt);
  const char* ab = static_cast<const char*>(a);
  const char* bb = static_cast<const char*>(b);
  if (ab < bb + bytes && bb < ab + bytes) return fail(DIAQ_ERR_INVALID_ARGUMENT, "state and scratch overlap");
  return DIAQ_OK;
}

}  // namespace

// Forward pass over gates[begin, end); *result receives the buffer that holds
// the final state (state or scratch).
diaq_status_t run_plain(diaq_ctx* ctx, const Prepared& p, int64_t begin, int64_t end, int n, diaq_dtype_t dt,
                        void* state, void* scratch, void** result) {
  DIAQ_TRY(ensure(ctx, &ctx->diag, size_t(p.max_values + workspace_slack(ctx, dt)) * elem_bytes(dt)));
  void* x = state;
  void* y = scratch;
  for (int64_t g = begin; g < end; g++) DIAQ_TRY(step(ctx, p.lg[g], p.offs[g], n, dt, false, &x, &y));
  *result = x;
  return DIAQ_OK;
}

// Fused forward pass: one expansion + product per planned op.
diaq_status_t run_fused(diaq_ctx* ctx, const std::vector<FusedOp>& ops, int n, diaq_dtype_t dt, void* state,
                        void* scratch, void** result) {
  std::vector<std::vector<int64_t>> offs(ops.size());
  OpTables tabs;
  int64_t max_values = 0;
  for (size_t k = 0; k < ops.size(); k++) {
    offs[k] = gate_offsets(ops[k].core);
    if (offs[k].size() > size_t(kMaxArgDiags))
      return fail(DIAQ_ERR_UNSUPPORTED, "fused op %zu has %zu diagonals", k, offs[k].size());
    max_values = std::max<int64_t>(max_values, packing_starts(offs[k], n).back());
    tabs.add(ops[k].post);
  }
  DIAQ_TRY(ensure(ctx, &ctx->diag, size_t(max_values + workspace_slack(ctx, dt)) * elem_bytes(dt)));
  const char* dtab = nullptr;
  if (!tabs.bytes.empty()) {
    DIAQ_TRY(ensure(ctx, &ctx->aux, tabs.bytes.size()));
    dtab = static_cast<const char*>(ctx->aux.ptr);
    DIAQ_TRY(upload(ctx, ctx->aux.ptr, tabs.bytes.data(), tabs.bytes.size()));
  }
  void* x = state;
  void* y = scratch;
  for (size_t k = 0; k < ops.size(); k++) {
    const int nt = tabs.count[k];
    DIAQ_TRY(step(ctx, ops[k].core, offs[k], n, dt, false, &x, &y, nt ? dtab + tabs.first[k] : nullptr, nt));
  }
  *result = x;
  return DIAQ_OK;
}

// Alg. 3 forward pass: every op applied in place on `state`, no expansion.
// Operations on the lowest qubits are staged through LDS as dense groups.
diaq_status_t run_kron(diaq_ctx* ctx, const std::vector<FusedOp>& ops, int n, diaq_dtype_t dt, void* state) {
  struct Staged {
    int S[6];
    int k = 0;
    size_t moff = 0;
  };
  std::vector<Staged> stg(ops.size());
  std::vector<double> mats, m;
  OpTables tabs;
  for (size_t k = 0; k < ops.size(); k++) {
    if (staged_dense(ops[k].core, n, int(ops[k].post.size()), ctx->tuning, dt, &m, stg[k].S, &stg[k].k)) {
      stg[k].moff = mats.size();
      mats.insert(mats.end(), m.begin(), m.end());
      tabs.add(ops[k].post);
    } else {
      // per-coset kernel: table headers carry the rows' index bits
      int64_t off[8];
      kron_row_offsets(ops[k].core, off);
      tabs.add(ops[k].post, off, 1 << ops[k].core.k);
    }
  }
  const size_t mb = ((mats.size() * sizeof(double) + 255) / 256) * 256;
  char* base = nullptr;
  if (mb + tabs.bytes.size()) {
    DIAQ_TRY(ensure(ctx, &ctx->aux, mb + tabs.bytes.size()));
    base = static_cast<char*>(ctx->aux.ptr);
    DIAQ_TRY(upload(ctx, base, mats.data(), mats.size() * sizeof(double)));
    DIAQ_TRY(upload(ctx, base + mb, tabs.bytes.data(), tabs.bytes.size()));
  }
  const double full = 2.0 * double(elem_bytes(dt)) * double(int64_t(1) << n);
  for (size_t k = 0; k < ops.size(); k++) {
    const int nt = tabs.count[k];
    const char* tk = nt ? base + mb + tabs.first[k] : nullptr;
    const size_t e0 = prof_mark(ctx);
    if (stg[k].k) {
      DIAQ_TRY(launch_staged(ctx, stg[k].S, stg[k].k, reinterpret_cast<const double*>(base) + stg[k].moff, tk, nt, n,
                             dt, state));
      prof_interval(ctx, e0, prof_mark(ctx), 1, full);
    } else {
      DIAQ_TRY(launch_kron_apply(ctx, ctx->stream, ops[k].core, n, dt, state, false, tk, nt, nullptr, true));
      prof_interval(ctx, e0, prof_mark(ctx), 1, kron_op_bytes(ops[k].core, int(ops[k].post.size()), n, dt));
    }
  }
  return DIAQ_OK;
}

std::vector<FusedOp> unfused_ops(const Prepared& p) {
  std::vector<FusedOp> ops(p.lg.size());
  for (size_t k = 0; k < p.lg.size(); k++) {
    ops[k].core = p.lg[k];
    ops[k].ngates = 1;
  }
  return ops;
}

// gates[begin, end) applied to `state` on ctx->stream; arguments checked.
diaq_status_t apply_range(diaq_ctx* ctx, const diaq_gate_t* gates, int64_t begin, int64_t end, int nqubits,
                          diaq_dtype_t dtype, void* state, void* scratch, const diaq_plan_t* plan) {
  const int saved_rows = ctx->spmv_rows;
  if (plan && plan->rows_per_thread) ctx->spmv_rows = plan->rows_per_thread;
  void* res = nullptr;
  diaq_status_t st;
  const int kmax = plan && plan->max_fused_qubits ? plan->max_fused_qubits : 2;
  if (plan && plan->kron && nqubits <= small_circuit_qubits(ctx, dtype)) {
    // a small state: the whole range in LDS, one launch per run of gates
    // (fusion buys nothing when no gate touches memory)
    Prepared p;
    st = prepare_gates(gates + begin, end - begin, nqubits, &p);
    if (st == DIAQ_OK) st = run_small(ctx, p.lg, nqubits, dtype, state);
    res = state;
  } else if (plan && plan->kron && plan->fuse && kmax > 3) {
    // groups of four or five qubits: dense local matrices
    std::vector<BigOp> ops;
    st = plan_big(gates + begin, end - begin, nqubits, kmax, &ops, dtype);
    if (st == DIAQ_OK) st = run_big(ctx, ops, nqubits, dtype, state);
    res = state;
  } else if (plan && plan->kron) {
    std::vector<FusedOp> ops;
    if (plan->fuse) {
      st = plan_fusion(gates + begin, end - begin, nqubits, kmax, dtype, &ops, true);
    } else {
      Prepared p;
      st = prepare_gates(gates + begin, end - begin, nqubits, &p);
      if (st == DIAQ_OK) ops = unfused_ops(p);
    }
    if (st == DIAQ_OK) st = run_kron(ctx, ops, nqubits, dtype, state);
    res = state;
  } else if (plan && plan->fuse) {
    std::vector<FusedOp> ops;
    st = plan_fusion(gates + begin, end - begin, nqubits, kmax, dtype, &ops);
    if (st == DIAQ_OK) st = run_fused(ctx, ops, nqubits, dtype, state, scratch, &res);
  } else {
    Prepared p;
    st = prepare_gates(gates + begin, end - begin, nqubits, &p);
    if (st == DIAQ_OK) st = run_plain(ctx, p, 0, end - begin, nqubits, dtype, state, scratch, &res);
  }
  ctx->spmv_rows = saved_rows;
  DIAQ_TRY(st);
  if (res != state)
    DIAQ_TRY(launch_copy(ctx->stream, res, state, (size_t(1) << nqubits) * elem_bytes(dtype)));
  return DIAQ_OK;
}

}  // namespace diaq

using namespace diaq;

extern "C" {

diaq_status_t diaq_apply_circuit(diaq_ctx_t ctx, const diaq_gate_t* gates, int64_t ngates, int64_t begin,
                                 int64_t end, int32_t nqubits, diaq_dtype_t dtype, void* state, void* scratch,
                                 const diaq_plan_t* plan) {
  try {
    if (!ctx) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (ngates < 0 || (ngates > 0 && !gates)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad gate list");
    if (begin < 0 || end < begin || end > ngates)
      return fail(DIAQ_ERR_INVALID_ARGUMENT, "gate range [%lld, %lld) outside [0, %lld]", (long long)begin,
                  (long long)end, (long long)ngates);
    DIAQ_TRY(check_vectors(nqubits, dtype, state, scratch));
    if (plan && plan->block != 0 && plan->block != 256)
      return fail(DIAQ_ERR_INVALID_ARGUMENT, "plan.block %d: the kernels use 256-lane workgroups", plan->block);
    return apply_range(ctx, gates, begin, end, nqubits, dtype, state, scratch, plan);
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

diaq_status_t diaq_copy(diaq_ctx_t ctx, const void* src, void* dst, size_t bytes) {
  if (!ctx || (bytes && (!src || !dst))) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
  return launch_copy(ctx->stream, src, dst, bytes);
}

diaq_status_t diaq_plan_count(const diaq_gate_t* gates, int64_t ngates, int32_t nqubits, diaq_dtype_t dtype,
                              const diaq_plan_t* plan, int64_t* nops, double* bytes) {
  try {
    if (ngates < 0 || (ngates > 0 && !gates)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad gate list");
    if (dtype != DIAQ_C64 && dtype != DIAQ_C128) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad dtype");
    const double s = double(elem_bytes(dtype)), N = double(int64_t(1) << nqubits);
    double b = 0;
    int64_t count = 0;
    if (plan && plan->kron && plan->fuse && plan->max_fused_qubits > 3) {
      std::vector<BigOp> ops;
      DIAQ_TRY(plan_big(gates, ngates, nqubits, plan->max_fused_qubits, &ops, dtype));
      count = int64_t(ops.size());
      b = double(count) * 2.0 * s * N;  // every operation reads and writes the state once
    } else if (plan && plan->kron) {
      if (plan->fuse) {
        std::vector<FusedOp> ops;
        DIAQ_TRY(plan_fusion(gates, ngates, nqubits, plan->max_fused_qubits ? plan->max_fused_qubits : 2, dtype,
                             &ops, true));
        count = int64_t(ops.size());
        for (const auto& op : ops) b += kron_op_bytes(op.core, int(op.post.size()), nqubits, dtype);
      } else {
        Prepared p;
        DIAQ_TRY(prepare_gates(gates, ngates, nqubits, &p));
        count = ngates;
        for (const auto& lg : p.lg) b += kron_op_bytes(lg, 0, nqubits, dtype);
      }
    } else if (plan && plan->fuse) {
      std::vector<FusedOp> ops;
      DIAQ_TRY(plan_fusion(gates, ngates, nqubits, plan->max_fused_qubits ? plan->max_fused_qubits : 2, dtype,
                           &ops));
      for (const auto& op : ops) b += s * (2.0 * double(packing_starts(gate_offsets(op.core), nqubits).back()) + 2 * N);
      count = int64_t(ops.size());
    } else {
      Prepared p;
      DIAQ_TRY(prepare_gates(gates, ngates, nqubits, &p));
      for (const auto& o : p.offs) b += s * (2.0 * double(packing_starts(o, nqubits).back()) + 2 * N);
      count = ngates;
    }
    if (nops) *nops = count;
    if (bytes) *bytes = b;
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

diaq_status_t diaq_adjoint_grad(diaq_ctx_t ctx, const diaq_gate_t* gates, int64_t ngates, int32_t nqubits,
                                diaq_dtype_t dtype, diaq_dia_t H, const void* psi0, void* work, int64_t nparams,
                                double* expval, double* grad, const diaq_plan_t* plan) {
  try {
    if (!ctx || !H || !psi0 || !work || !expval || (nparams > 0 && !grad))
      return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
    if (ngates < 0 || (ngates > 0 && !gates)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad gate list");
    if (H->nqubits != nqubits || H->dtype != dtype)
      return fail(DIAQ_ERR_NOT_MULTIPLYABLE, "observable is 2^%d, register 2^%d", H->nqubits, nqubits);
    const size_t N = size_t(1) << nqubits;
    const size_t vb = N * elem_bytes(dtype);
    char* w = static_cast<char*>(work);
    void* psi = w;
    void* lam = w + vb;
    void* tmp = w + 2 * vb;
    DIAQ_TRY(check_vectors(nqubits, dtype, psi, lam));
    {
      const char* p0 = static_cast<const char*>(psi0);
      if (p0 < w + 3 * vb && w < p0 + vb) return fail(DIAQ_ERR_INVALID_ARGUMENT, "psi0 overlaps work");
    }
    Prepared p;
    DIAQ_TRY(prepare_gates(gates, ngates, nqubits, &p));
    std::vector<LocalGate> gens(static_cast<size_t>(ngates));
    std::vector<int> diff(static_cast<size_t>(ngates), 0);
    for (int64_t g = 0; g < ngates; g++) {
      if (gates[g].param_index < 0) continue;
      if (gates[g].param_index >= nparams)
        return fail(DIAQ_ERR_INVALID_ARGUMENT, "gate %lld: param_index %d >= nparams %lld", (long long)g,
                    gates[g].param_index, (long long)nparams);
      gens[g] = p.lg[g];
      if (!local_generator(&gates[g], &gens[g]))
        return fail(DIAQ_ERR_UNSUPPORTED, "gate %lld: kind %d is not a rotation with a generator", (long long)g,
                    gates[g].kind);
      diff[g] = 1;
    }
    const bool kron = plan && plan->kron;
    // forward: psi = U psi0 (Alg. 3 plan: fused in-place operations)
    DIAQ_TRY(launch_copy(ctx->stream, psi0, psi, vb));
    if (kron) {
      const int kmax = plan->max_fused_qubits > 0 ? plan->max_fused_qubits : 4;
      if (kmax > 3) {
        std::vector<BigOp> ops;
        DIAQ_TRY(plan_big(gates, ngates, nqubits, kmax, &ops, dtype));
        DIAQ_TRY(run_big(ctx, ops, nqubits, dtype, psi));
      } else {
        std::vector<FusedOp> ops;
        DIAQ_TRY(plan_fusion(gates, ngates, nqubits, kmax, dtype, &ops, true));
        DIAQ_TRY(run_kron(ctx, ops, nqubits, dtype, psi));
      }
    } else {
      void* res = nullptr;
      DIAQ_TRY(run_plain(ctx, p, 0, ngates, nqubits, dtype, psi, tmp, &res));
      if (res != psi) std::swap(psi, tmp);
    }
    // Alg. 3 reverse sweep: segments of gates per pass (n >= 3)
    const bool segmented = kron && nqubits >= 3;
    SegmentPlan sp;
    std::vector<char> table;
    if (segmented) {
      // dot keys: gates with the same parameter and scale may share a dot
      std::vector<int64_t> dkey(size_t(ngates), -1);
      std::map<std::pair<int32_t, double>, int64_t> keys;
      for (int64_t g = 0; g < ngates; g++)
        if (diff[size_t(g)]) {
          const auto k = std::make_pair(gates[g].param_index, gates[g].param_scale);
          auto it = keys.find(k);
          if (it == keys.end()) {
            const int64_t id = int64_t(keys.size());
            it = keys.emplace(k, id).first;
          }
          dkey[size_t(g)] = it->second;
        }
      DIAQ_TRY(plan_segments(p.lg, gens, dkey, nqubits, &sp));
      std::vector<int64_t> slots(sp.dot_gate.size());
      for (size_t j = 0; j < slots.size(); j++) slots[j] = sp.dot_gate[j] + 1;
      segment_table_host(sp, table, slots);
    }
    // device slots: [0] = <psi|H|psi>, [1 + g] = <lam|G_g|psi>; the segment
    // table follows
    const size_t dots_bytes = ((size_t(ngates + 1) * 2 * sizeof(double) + 255) / 256) * 256;
    DIAQ_TRY(ensure(ctx, &ctx->aux, dots_bytes + table.size() + 256));
    double* dots = static_cast<double*>(ctx->aux.ptr);
    char* dtable = static_cast<char*>(ctx->aux.ptr) + dots_bytes;
    DIAQ_HIP(hipMemsetAsync(dots, 0, size_t(ngates + 1) * 2 * sizeof(double), ctx->stream));
    if (segmented) {
      // per-segment partial sums, reduced in one launch after the sweep; the
      // reduce records point into this buffer, so it is sized here for the
      // generator dot below too (which must not reallocate it)
      const int64_t rows = std::max<int64_t>(segment_partial_entries(sp, nqubits), (int64_t(1) << nqubits) / 256 + 1);
      DIAQ_TRY(ensure(ctx, &ctx->red, size_t(rows) * sizeof(double2)));
      segment_table_reds(sp, nqubits, dtable, static_cast<const double2*>(ctx->red.ptr), table);
    }
    if (!table.empty()) {
      // synchronous: the host image dies with this call
      DIAQ_HIP(hipStreamSynchronize(ctx->stream));
      DIAQ_HIP(hipMemcpy(dtable, table.data(), table.size(), hipMemcpyHostToDevice));
    }
    // lam = H psi ; E = <psi|lam>
    DIAQ_TRY(launch_spmv(ctx, op_of(H, H->transposed, H->conjugated), psi, lam));
    LocalGate ident;
    std::memset(&ident, 0, sizeof(ident));
    ident.k = 1;
    ident.targets[0] = 0;
    ident.m[0][0][0] = 1;
    ident.m[1][1][0] = 1;
    DIAQ_TRY(launch_generator_dot(ctx, ident, nqubits, dtype, psi, lam, dots));
    // reverse sweep
    if (segmented) {
      DIAQ_TRY(run_segments(ctx, ctx->stream, sp, nqubits, dtype, psi, lam, dtable,
                            static_cast<double2*>(ctx->red.ptr), dots));
    } else if (kron) {
      // one fused Alg. 3 pass per gate: generator dot, then psi, lam <- U^dagger
      int64_t maxb = 1;
      for (int64_t g = 0; g < ngates; g++) maxb = std::max(maxb, kron_adjoint_blocks(p.lg[g], nqubits));
      DIAQ_TRY(ensure(ctx, &ctx->red, size_t(maxb) * sizeof(double2)));
      double2* partial = static_cast<double2*>(ctx->red.ptr);
      for (int64_t g = ngates - 1; g >= 0; g--) {
        if (!diff[g] && g == 0) break;
        DIAQ_TRY(launch_kron_adjoint(ctx, ctx->stream, p.lg[g], diff[g] ? &gens[g] : nullptr, nqubits, dtype, psi,
                                     lam, partial, g > 0));
        if (diff[g])
          DIAQ_TRY(launch_final_reduce(ctx->stream, partial, kron_adjoint_blocks(p.lg[g], nqubits),
                                       dots + 2 * (g + 1)));
      }
    } else {
      for (int64_t g = ngates - 1; g >= 0; g--) {
        if (diff[g]) DIAQ_TRY(launch_generator_dot(ctx, gens[g], nqubits, dtype, lam, psi, dots + 2 * (g + 1)));
        if (g == 0) break;
        DIAQ_TRY(step(ctx, p.lg[g], p.offs[g], nqubits, dtype, true, &psi, &tmp));
        DIAQ_TRY(step(ctx, p.lg[g], p.offs[g], nqubits, dtype, true, &lam, &tmp));
      }
    }
    const size_t rb = size_t(ngates + 1) * 2 * sizeof(double);
    DIAQ_TRY(ensure_pinned(ctx, rb));
    DIAQ_HIP(hipMemcpyAsync(ctx->pinned, dots, rb, hipMemcpyDeviceToHost, ctx->stream));
    DIAQ_HIP(hipStreamSynchronize(ctx->stream));
    *expval = ctx->pinned[0];
    for (int64_t j = 0; j < nparams; j++) grad[j] = 0.0;
    for (int64_t g = 0; g < ngates; g++)
      if (diff[g]) grad[gates[g].param_index] += gates[g].param_scale * ctx->pinned[2 * (g + 1) + 1];
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Circuit graphs: one application of a gate list recorded once and replayed
// ---------------------------------------------------------------------------

struct diaq_graph {
  int device = 0;
  diaq::Workspace diag, aux, red;  // owned: other calls never touch them
  char* host = nullptr;            // pinned tables the replay copies in
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t nodes = 0;
};

namespace {

void release_graph(diaq_graph* G) {
  if (!G) return;
  if (G->exec) (void)hipGraphExecDestroy(G->exec);
  if (G->g) (void)hipGraphDestroy(G->g);
  if (G->diag.ptr) (void)hipFree(G->diag.ptr);
  if (G->aux.ptr) (void)hipFree(G->aux.ptr);
  if (G->red.ptr) (void)hipFree(G->red.ptr);
  if (G->host) (void)hipHostFree(G->host);
  delete G;
}

diaq_status_t alloc_exact(Workspace* w) {
  if (w->want == 0) return DIAQ_OK;
  const hipError_t e = hipMalloc(&w->ptr, w->want);
  if (e != hipSuccess) {
    w->ptr = nullptr;
    (void)hipGetLastError();
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "hipMalloc(%zu bytes) for a circuit graph: %s", w->want,
                hipGetErrorString(e));
  }
  w->bytes = w->want;
  return DIAQ_OK;
}

// Record apply_range on `cs` with the graph's workspaces swapped into the
// context.  The context is restored whatever happens.
diaq_status_t record(diaq_ctx* ctx, diaq_graph* G, Capture* cap, hipStream_t cs, const diaq_gate_t* gates,
                     int64_t ngates, int nqubits, diaq_dtype_t dtype, void* state, void* scratch,
                     const diaq_plan_t* plan, hipGraph_t* out) {
  std::swap(ctx->diag, G->diag);
  std::swap(ctx->aux, G->aux);
  std::swap(ctx->red, G->red);
  const hipStream_t saved_stream = ctx->stream;
  const bool saved_prof = ctx->profiling;
  ctx->stream = cs;
  ctx->profiling = false;
  ctx->capture = cap;
  diaq_status_t st = DIAQ_OK;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    st = fail(DIAQ_ERR_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  } else {
    st = apply_range(ctx, gates, 0, ngates, nqubits, dtype, state, scratch, plan);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (st == DIAQ_OK && e != hipSuccess)
      st = fail(DIAQ_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (st == DIAQ_OK) {
      *out = g;
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  (void)hipGetLastError();
  ctx->capture = nullptr;
  ctx->profiling = saved_prof;
  ctx->stream = saved_stream;
  std::swap(ctx->diag, G->diag);
  std::swap(ctx->aux, G->aux);
  std::swap(ctx->red, G->red);
  return st;
}

}  // namespace

extern "C" {

diaq_status_t diaq_circuit_graph_create(diaq_ctx_t ctx, const diaq_gate_t* gates, int64_t ngates, int32_t nqubits,
                                        diaq_dtype_t dtype, void* state, void* scratch, const diaq_plan_t* plan,
                                        diaq_graph_t* out) {
  if (!out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx is NULL");
  if (ctx->capture) return fail(DIAQ_ERR_INVALID_ARGUMENT, "the context is already recording a graph");
  if (ngates < 0 || (ngates > 0 && !gates)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad gate list");
  DIAQ_TRY(check_vectors(nqubits, dtype, state, scratch));
  if (plan && plan->block != 0 && plan->block != 256)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "plan.block %d: the kernels use 256-lane workgroups", plan->block);
  diaq_graph* G = nullptr;
  hipStream_t cs = nullptr;
  try {
    G = new diaq_graph;
    G->device = ctx->device;
    // the legacy stream cannot be recorded: a private stream of default
    // priority carries the recording
    const hipError_t ce = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (ce != hipSuccess) {
      (void)hipGetLastError();
      release_graph(G);
      return fail(DIAQ_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(ce));
    }
    Capture cap;
    hipGraph_t g = nullptr;
    diaq_status_t st = record(ctx, G, &cap, cs, gates, ngates, nqubits, dtype, state, scratch, plan, &g);
    if (st == DIAQ_OK) {
      (void)hipGraphDestroy(g);
      g = nullptr;
      st = alloc_exact(&G->diag);
      if (st == DIAQ_OK) st = alloc_exact(&G->aux);
      if (st == DIAQ_OK) st = alloc_exact(&G->red);
      if (st == DIAQ_OK && cap.host_used) {
        if (hipHostMalloc(reinterpret_cast<void**>(&G->host), cap.host_used, hipHostMallocDefault) != hipSuccess) {
          G->host = nullptr;
          (void)hipGetLastError();
          st = fail(DIAQ_ERR_OUT_OF_MEMORY, "pinned staging of %zu bytes", cap.host_used);
        }
      }
    }
    if (st == DIAQ_OK) {
      cap.sizing = false;
      cap.host = G->host;
      cap.host_bytes = cap.host_used;
      cap.host_used = 0;
      st = record(ctx, G, &cap, cs, gates, ngates, nqubits, dtype, state, scratch, plan, &g);
    }
    if (st == DIAQ_OK) {
      G->g = g;
      size_t nn = 0;
      if (hipGraphGetNodes(g, nullptr, &nn) == hipSuccess) G->nodes = int64_t(nn);
      const hipError_t ie = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        G->exec = nullptr;
        (void)hipGetLastError();
        st = fail(DIAQ_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
      }
    }
    (void)hipStreamDestroy(cs);
    if (st != DIAQ_OK) {
      release_graph(G);
      return st;
    }
    *out = G;
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    if (cs) (void)hipStreamDestroy(cs);
    release_graph(G);
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

diaq_status_t diaq_circuit_graph_launch(diaq_ctx_t ctx, diaq_graph_t graph) {
  if (!ctx || !graph) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL context or graph");
  if (graph->device != ctx->device)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "graph of device %d launched from a context of device %d", graph->device,
                ctx->device);
  if (ctx->capture) return fail(DIAQ_ERR_INVALID_ARGUMENT, "the context is recording a graph");
  DIAQ_HIP(hipGraphLaunch(graph->exec, ctx->stream));
  return DIAQ_OK;
}

diaq_status_t diaq_circuit_graph_nodes(diaq_graph_t graph, int64_t* nodes) {
  if (!graph || !nodes) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL graph or output");
  *nodes = graph->nodes;
  return DIAQ_OK;
}

diaq_status_t diaq_circuit_graph_free(diaq_graph_t graph) {
  if (!graph) return DIAQ_OK;
  // a replay still in flight reads the graph's workspaces
  DIAQ_HIP(hipDeviceSynchronize());
  release_graph(graph);
  return DIAQ_OK;
}

}  // extern "C"

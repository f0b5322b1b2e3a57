// autotune.cpp -- picks the product kernel's knobs and a circuit's plan by
// measurement, with a JSON cache for the kernel knobs.
//
// The paper's cost model (Sec. IV: O(N d) for a product, O(d1 d2 N) for a
// matrix product) says how much work a plan does; on an HBM-bound GPU the
// time follows the bytes, so plans are ranked by their algorithmic bytes
// and the best few are timed.
#include <cstdio>
#include <string>

#include "internal.hpp"

namespace diaq {

namespace {

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// The key names the architecture and compute-unit count; the marketing
// name is left out because some tool environments report it empty.
std::string device_name(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string s = p.gcnArchName;
  for (char& c : s)
    if (c == '"' || c == '\\' || c == '\n') c = ' ';
  return s + "/cu" + std::to_string(p.multiProcessorCount);
}

std::string cache_key(int dev, int n, diaq_dtype_t dt) {
  return device_name(dev) + "|n=" + std::to_string(n) + "|" + (dt == DIAQ_C128 ? "c128" : "c64");
}

std::string read_file(const char* path) {
  std::string s;
  FILE* f = std::fopen(path, "rb");
  if (!f) return s;
  char buf[4096];
  size_t r;
  while ((r = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, r);
  std::fclose(f);
  return s;
}

bool u64_field(const std::string& obj, const char* name, uint64_t* v) {
  const std::string pat = std::string("\"") + name + "\":";
  size_t p = obj.find(pat);
  if (p == std::string::npos) return false;
  *v = std::strtoull(obj.c_str() + p + pat.size(), nullptr, 10);
  return true;
}

bool int_field(const std::string& obj, const char* name, int32_t* v) {
  const std::string pat = std::string("\"") + name + "\":";
  size_t p = obj.find(pat);
  if (p == std::string::npos) return false;
  *v = int32_t(std::strtol(obj.c_str() + p + pat.size(), nullptr, 10));
  return true;
}

// Entries are one JSON object per line inside {"entries": [ ... ]}.
bool cache_lookup(const char* path, const std::string& key, diaq_tuning_t* t) {
  const std::string text = read_file(path);
  const std::string pat = "\"key\":\"" + key + "\"";
  size_t p = text.find(pat);
  if (p == std::string::npos) return false;
  const size_t b = text.rfind('{', p), e = text.find('}', p);
  if (b == std::string::npos || e == std::string::npos) return false;
  const std::string obj = text.substr(b, e - b + 1);
  diaq_tuning_t r{};
  bool ok = int_field(obj, "spmv_rows", &r.spmv_rows) && int_field(obj, "spmv_group_bits", &r.spmv_group_bits) &&
            int_field(obj, "spmv_chunk", &r.spmv_chunk) && int_field(obj, "spmv_nontemporal", &r.spmv_nontemporal) &&
            int_field(obj, "spmv_group_min_qubit", &r.spmv_group_min_qubit);
  if (ok) u64_field(obj, "spmv_group_qubits", &r.spmv_group_qubits);
  if (ok) *t = r;
  return ok;
}

diaq_status_t cache_store(const char* path, const std::string& key, const diaq_tuning_t& t, double ms) {
  const std::string text = read_file(path);
  std::vector<std::string> lines;
  size_t p = 0;
  while (true) {
    const size_t b = text.find("{\"key\":", p);
    if (b == std::string::npos) break;
    const size_t e = text.find('}', b);
    if (e == std::string::npos) break;
    const std::string obj = text.substr(b, e - b + 1);
    if (obj.find("\"key\":\"" + key + "\"") == std::string::npos) lines.push_back(obj);
    p = e + 1;
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "{\"key\":\"%s\",\"spmv_rows\":%d,\"spmv_group_bits\":%d,\"spmv_chunk\":%d,"
                "\"spmv_nontemporal\":%d,\"spmv_group_min_qubit\":%d,\"spmv_group_qubits\":%llu,\"ms\":%.4f}",
                key.c_str(), t.spmv_rows, t.spmv_group_bits, t.spmv_chunk, t.spmv_nontemporal,
                t.spmv_group_min_qubit, (unsigned long long)t.spmv_group_qubits, ms);
  lines.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(DIAQ_ERR_INVALID_ARGUMENT, "cannot write autotune cache %s", tmp.c_str());
  std::fprintf(f, "{\"entries\": [\n");
  for (size_t i = 0; i < lines.size(); i++) std::fprintf(f, "  %s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
  std::fprintf(f, "]}\n");
  std::fclose(f);
  if (std::rename(tmp.c_str(), path) != 0) return fail(DIAQ_ERR_INVALID_ARGUMENT, "cannot replace %s", path);
  return DIAQ_OK;
}

std::vector<diaq_tuning_t> candidates() {
  std::vector<diaq_tuning_t> c;
  for (int rows : {1, 2, 4})
    for (int chunk : {1, 3})
      for (int nt : {1, -1})
        for (int gmin : {19, 21, 23, 0}) {
          diaq_tuning_t t{};
          t.spmv_rows = rows;
          t.spmv_chunk = chunk;
          t.spmv_nontemporal = nt;
          t.spmv_group_bits = gmin ? 0 : -1;  // 0: up to 3 paired qubits; -1: none
          t.spmv_group_min_qubit = gmin ? gmin : 0;
          c.push_back(t);
        }
  return c;
}

// The candidate with the product kernel's built-in shape (one row per lane,
// one diagonal per chunk, non-temporal streams, pairing from qubit 21).
diaq_tuning_t tune_default() {
  diaq_tuning_t t{};
  t.spmv_rows = 1;
  t.spmv_chunk = 1;
  t.spmv_nontemporal = 1;
  t.spmv_group_bits = 0;
  t.spmv_group_min_qubit = 21;
  return t;
}
const diaq_tuning_t kTuneDefault = tune_default();

// The SpMV autotuner chooses the product-kernel knobs only; the others
// (expansion, workspace padding, Alg. 3 kernels) keep their current values.
void keep_other_knobs(const diaq_tuning_t& cur, diaq_tuning_t* best) {
  best->expand_nontemporal = cur.expand_nontemporal;
  best->diag_pad = cur.diag_pad;
  best->kron_stage_qubit = cur.kron_stage_qubit;
  best->kron_split = cur.kron_split;
  best->kron_nontemporal = cur.kron_nontemporal;
  best->kron_small_qubits = cur.kron_small_qubits;
  best->kron_order = cur.kron_order;
  best->spmv_order = cur.spmv_order;
  best->spmv_pack = cur.spmv_pack;
}

}  // namespace

}  // namespace diaq

using namespace diaq;

extern "C" {

diaq_status_t diaq_autotune(diaq_ctx_t ctx, int32_t nqubits, diaq_dtype_t dtype, const char* cache_path,
                            diaq_tuning_t* out) {
  try {
    if (!ctx) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (nqubits < 1 || nqubits > 32) return fail(DIAQ_ERR_INVALID_ARGUMENT, "nqubits %d out of range", nqubits);
    if (dtype != DIAQ_C64 && dtype != DIAQ_C128) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad dtype");
    const std::string key = cache_key(ctx->device, nqubits, dtype);
    diaq_tuning_t best{};
    if (cache_path && cache_lookup(cache_path, key, &best)) {
      keep_other_knobs(ctx->tuning, &best);
      ctx->tuning = best;
      if (out) *out = best;
      return DIAQ_OK;
    }
    const int n = nqubits;
    const size_t N = size_t(1) << n, s = elem_bytes(dtype);
    // test gates: U3 on qubits spread over the register, and one CX
    std::vector<diaq_gate_t> gates;
    std::vector<int> qs = {0, n / 3, (2 * n) / 3, n - 1};
    std::sort(qs.begin(), qs.end());
    qs.erase(std::unique(qs.begin(), qs.end()), qs.end());
    for (int q : qs) {
      diaq_gate_t g{};
      g.kind = DIAQ_GATE_U3;
      g.ntargets = 1;
      g.targets[0] = q;
      g.params[0] = 0.3;
      g.params[1] = 0.5;
      g.params[2] = 0.7;
      g.param_index = -1;
      gates.push_back(g);
    }
    if (n >= 2) {
      diaq_gate_t g{};
      g.kind = DIAQ_GATE_X;
      g.ntargets = 1;
      g.ncontrols = 1;
      g.targets[0] = n / 2;
      g.controls[0] = n / 2 - 1 >= 0 ? n / 2 - 1 : n / 2 + 1;
      g.param_index = -1;
      gates.push_back(g);
    }
    void* x = nullptr;
    void* y = nullptr;
    DIAQ_HIP(hipMalloc(&x, N * s));
    if (hipMalloc(&y, N * s) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(x);
      return fail(DIAQ_ERR_OUT_OF_MEMORY, "autotune vectors");
    }
    struct Free {
      void* a;
      void* b;
      ~Free() {
        (void)hipFree(a);
        (void)hipFree(b);
      }
    } guard{x, y};
    DIAQ_HIP(hipMemsetAsync(x, 0, N * s, ctx->stream));
    const diaq_tuning_t saved = ctx->tuning;
    const std::vector<diaq_tuning_t> cand = candidates();
    double best_ms = 0;
    Timer tm;
    const int reps = n >= 24 ? 3 : 10;
    // time of candidate c on the expanded test gate `op` (one warm-up launch)
    auto time_one = [&](const SpmvOp& op, const diaq_tuning_t& t, int launches, double* ms_out) -> diaq_status_t {
      ctx->tuning = t;
      DIAQ_TRY(launch_spmv(ctx, op, x, y));
      DIAQ_HIP(hipEventRecord(tm.a, ctx->stream));
      for (int r = 0; r < launches; r++) DIAQ_TRY(launch_spmv(ctx, op, x, y));
      DIAQ_HIP(hipEventRecord(tm.b, ctx->stream));
      DIAQ_HIP(hipEventSynchronize(tm.b));
      float ms = 0;
      DIAQ_HIP(hipEventElapsedTime(&ms, tm.a, tm.b));
      *ms_out = ms / launches;
      return DIAQ_OK;
    };
    auto expand_test_gate = [&](const diaq_gate_t& g, std::vector<int64_t>* offs, std::vector<int64_t>* st,
                                SpmvOp* op) -> diaq_status_t {
      LocalGate lg;
      DIAQ_TRY(local_gate(&g, n, &lg));
      *offs = gate_offsets(lg);
      *st = packing_starts(*offs, n);
      DIAQ_TRY(ensure(ctx, &ctx->diag, size_t(st->back()) * s));
      DIAQ_TRY(launch_expand(ctx, lg, n, dtype, *offs, *st, ctx->diag.ptr));
      op->n = n;
      op->dtype = dtype;
      op->nd = int(offs->size());
      op->host_off = offs->data();
      op->host_start = st->data();
      op->values = ctx->diag.ptr;
      op->qubit_mask = lg.tmask;
      op->skip_zero = true;
      return DIAQ_OK;
    };
    // Stage 1: the summed time over the test gates of every candidate; then
    // the six fastest and the default shape are timed in two more rounds and
    // ranked by their median round (the variants differ by a few per cent,
    // so one round can order them differently from box to box).  The
    // default shape is kept unless another beats it by more than 2 %.
    auto round_times = [&](const std::vector<size_t>& which, std::vector<double>* tot) -> diaq_status_t {
      tot->assign(which.size(), 0.0);
      for (const auto& g : gates) {
        std::vector<int64_t> offs, st;
        SpmvOp op;
        DIAQ_TRY(expand_test_gate(g, &offs, &st, &op));
        for (size_t w = 0; w < which.size(); w++) {
          double ms = 0;
          DIAQ_TRY(time_one(op, cand[which[w]], reps, &ms));
          (*tot)[w] += ms;
        }
      }
      return DIAQ_OK;
    };
    std::vector<size_t> all(cand.size());
    for (size_t c = 0; c < cand.size(); c++) all[c] = c;
    std::vector<double> first;
    DIAQ_TRY(round_times(all, &first));
    size_t def = 0;
    for (size_t c = 0; c < cand.size(); c++)
      if (cand[c].spmv_rows == kTuneDefault.spmv_rows && cand[c].spmv_chunk == kTuneDefault.spmv_chunk &&
          cand[c].spmv_nontemporal == kTuneDefault.spmv_nontemporal &&
          cand[c].spmv_group_min_qubit == kTuneDefault.spmv_group_min_qubit)
        def = c;
    std::vector<size_t> order = all;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return first[a] < first[b]; });
    std::vector<size_t> finalists(order.begin(), order.begin() + std::min<size_t>(6, order.size()));
    if (std::find(finalists.begin(), finalists.end(), def) == finalists.end()) finalists.push_back(def);
    std::vector<std::vector<double>> rounds(finalists.size());
    for (size_t w = 0; w < finalists.size(); w++) rounds[w].push_back(first[finalists[w]]);
    for (int r = 0; r < 2; r++) {
      std::vector<double> tot;
      DIAQ_TRY(round_times(finalists, &tot));
      for (size_t w = 0; w < finalists.size(); w++) rounds[w].push_back(tot[w]);
    }
    std::vector<double> med(finalists.size());
    size_t bw = 0, dw = 0;
    for (size_t w = 0; w < finalists.size(); w++) {
      std::vector<double> r = rounds[w];
      std::sort(r.begin(), r.end());
      med[w] = r[r.size() / 2];
      if (med[w] < med[bw]) bw = w;
      if (finalists[w] == def) dw = w;
    }
    const size_t bi = med[bw] < 0.98 * med[dw] ? finalists[bw] : def;
    best = cand[bi];
    best_ms = med[bi == def ? dw : bw];
    // Stage 2: tile pairing qubit by qubit: a U3 on q, timed unpaired and
    // paired in three alternating rounds (partner rows 2^q apart meet in the
    // caches for some q and not others); a qubit is paired only if the
    // median paired time is more than 3 % below the median unpaired one
    const int tile_log2 = 8 + (best.spmv_rows == 4 ? 2 : best.spmv_rows == 2 ? 1 : 0);
    if (n > tile_log2 + 1) {
      uint64_t mask = 0;
      for (int q = tile_log2; q < n; q++) {
        diaq_gate_t g{};
        g.kind = DIAQ_GATE_U3;
        g.ntargets = 1;
        g.targets[0] = q;
        g.params[0] = 0.3;
        g.params[1] = 0.5;
        g.params[2] = 0.7;
        g.param_index = -1;
        std::vector<int64_t> offs, st;
        SpmvOp op;
        DIAQ_TRY(expand_test_gate(g, &offs, &st, &op));
        std::vector<double> t2[2];
        for (int r = 0; r < 3; r++)
          for (int paired = 0; paired < 2; paired++) {
            diaq_tuning_t t = best;
            t.spmv_group_bits = paired ? 1 : -1;
            t.spmv_group_qubits = uint64_t(1) << q;
            double ms = 0;
            DIAQ_TRY(time_one(op, t, 2 * reps, &ms));
            t2[paired].push_back(ms);
          }
        for (auto& v : t2) std::sort(v.begin(), v.end());
        if (t2[1][1] < 0.97 * t2[0][1]) mask |= uint64_t(1) << q;  // a clear win only
      }
      best.spmv_group_bits = 0;
      // a mask of zero means "no per-qubit choice": keep one unused high bit
      best.spmv_group_qubits = mask ? mask : (uint64_t(1) << 63);
    }
    keep_other_knobs(saved, &best);
    ctx->tuning = best;
    if (cache_path) DIAQ_TRY(cache_store(cache_path, key, best, best_ms));
    if (out) *out = best;
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

diaq_status_t diaq_autotune_plan(diaq_ctx_t ctx, const diaq_gate_t* gates, int64_t ngates, int32_t nqubits,
                                 diaq_dtype_t dtype, int32_t allow_kron, int32_t measure, diaq_plan_t* out) {
  try {
    if (!ctx || !out || ngates < 0 || (ngates > 0 && !gates)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad arguments");
    if (nqubits < 1 || nqubits > 34) return fail(DIAQ_ERR_INVALID_ARGUMENT, "nqubits out of range");
    if (dtype != DIAQ_C64 && dtype != DIAQ_C128) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad dtype");
    const int n = nqubits;
    const double s = double(elem_bytes(dtype)), N = double(int64_t(1) << n);
    struct Cand {
      diaq_plan_t plan;
      double est_ms;
      double max_bytes;  // largest expanded operation
    };
    std::vector<Cand> cands;
    // measured-or-nominal rates (GB/s) for the byte model
    const double rate_dia = 6000.0, rate_kron = 5700.0, launch_ms = 0.004;
    auto add = [&](int fuse, int k, int kron) -> diaq_status_t {
      diaq_plan_t p{};
      p.fuse = fuse;
      p.max_fused_qubits = k;
      p.kron = kron;
      std::vector<FusedOp> ops;
      double bytes = 0, maxb = 0;
      int64_t nops = 0;
      if (kron && fuse && k > 3) {
        std::vector<BigOp> big;
        DIAQ_TRY(plan_big(gates, ngates, n, k, &big, dtype));
        nops = int64_t(big.size());
        bytes = double(nops) * 2.0 * s * N;
        cands.push_back(Cand{p, bytes / (rate_kron * 1e6) + double(nops) * launch_ms, 0.0});
        return DIAQ_OK;
      }
      if (fuse) {
        DIAQ_TRY(plan_fusion(gates, ngates, n, k, dtype, &ops, kron != 0));
      } else {
        ops.resize(size_t(ngates));
        for (int64_t g = 0; g < ngates; g++) {
          DIAQ_TRY(local_gate(&gates[g], n, &ops[size_t(g)].core));
          ops[size_t(g)].ngates = 1;
        }
      }
      for (const auto& op : ops) {
        const double E = double(packing_starts(gate_offsets(op.core), n).back());
        if (kron) {
          bytes += kron_op_bytes(op.core, int(op.post.size()), n, dtype);
        } else {
          bytes += s * (2 * E + 2 * N);
          maxb = std::max(maxb, s * E);
          if (gate_offsets(op.core).size() > size_t(kMaxArgDiags)) return DIAQ_OK;  // not runnable
        }
      }
      nops = int64_t(ops.size());
      const double est = bytes / ((kron ? rate_kron : rate_dia) * 1e6) + double(nops) * launch_ms;
      cands.push_back(Cand{p, est, maxb});
      return DIAQ_OK;
    };
    DIAQ_TRY(add(0, 0, 0));
    for (int k = 1; k <= 3; k++) DIAQ_TRY(add(1, k, 0));
    if (allow_kron) {
      DIAQ_TRY(add(0, 0, 1));
      for (int k = 1; k <= 5; k++) DIAQ_TRY(add(1, k, 1));
    }
    size_t free_b = 0, total_b = 0;
    DIAQ_HIP(hipMemGetInfo(&free_b, &total_b));
    const double avail = double(free_b) + double(ctx->diag.bytes) - 2 * s * N - double(64 << 20);
    std::vector<Cand> fit;
    for (const auto& c : cands)
      if (c.max_bytes <= avail) fit.push_back(c);
    if (fit.empty()) return fail(DIAQ_ERR_OUT_OF_MEMORY, "no plan fits in device memory");
    std::stable_sort(fit.begin(), fit.end(), [](const Cand& a, const Cand& b) { return a.est_ms < b.est_ms; });
    const size_t nm = std::min(fit.size(), size_t(std::max(0, measure)));
    if (nm <= 1 || ngates == 0) {
      *out = fit[0].plan;
      return DIAQ_OK;
    }
    // time the leaders on the circuit's first quarter (at least 64 gates):
    // a shorter prefix cuts wide groups short and favours narrow ones
    const int64_t ng = std::min<int64_t>(ngates, std::max<int64_t>(64, ngates / 4));
    void* st = nullptr;
    void* sc = nullptr;
    const size_t vb = size_t(N) * size_t(s);
    DIAQ_HIP(hipMalloc(&st, vb));
    if (hipMalloc(&sc, vb) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(st);
      return fail(DIAQ_ERR_OUT_OF_MEMORY, "autotune vectors");
    }
    struct Free {
      void* a;
      void* b;
      ~Free() {
        (void)hipFree(a);
        (void)hipFree(b);
      }
    } guard{st, sc};
    DIAQ_HIP(hipMemsetAsync(st, 0, vb, ctx->stream));
    Timer tm;
    double best = 1e300;
    size_t bi = 0;
    for (size_t c = 0; c < nm; c++) {
      DIAQ_TRY(diaq_apply_circuit(ctx, gates, ng, 0, ng, n, dtype, st, sc, &fit[c].plan));  // warm-up
      DIAQ_HIP(hipEventRecord(tm.a, ctx->stream));
      DIAQ_TRY(diaq_apply_circuit(ctx, gates, ng, 0, ng, n, dtype, st, sc, &fit[c].plan));
      DIAQ_HIP(hipEventRecord(tm.b, ctx->stream));
      DIAQ_HIP(hipEventSynchronize(tm.b));
      float ms = 0;
      DIAQ_HIP(hipEventElapsedTime(&ms, tm.a, tm.b));
      if (ms < best) {
        best = ms;
        bi = c;
      }
    }
    *out = fit[bi].plan;
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

}  // extern "C"

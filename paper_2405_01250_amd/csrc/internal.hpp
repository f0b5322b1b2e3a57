// internal.hpp -- shared declarations of libdiaq_hip (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <string>
#include <vector>

#include "diaq.h"

namespace diaq {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

diaq_status_t fail(diaq_status_t st, const char* fmt, ...);
void clear_error();

#define DIAQ_HIP(expr)                                                       \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::diaq::fail(e_ == hipErrorOutOfMemory ? DIAQ_ERR_OUT_OF_MEMORY \
                                                    : DIAQ_ERR_DEVICE,       \
                          "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

#define DIAQ_TRY(expr)                  \
  do {                                  \
    diaq_status_t s_ = (expr);          \
    if (s_ != DIAQ_OK) return s_;       \
  } while (0)

// ---------------------------------------------------------------------------
// Complex helpers (interleaved re/im, 8- or 16-byte elements)
// ---------------------------------------------------------------------------

template <typename R> struct Cx;
template <> struct Cx<double> { using V = double2; };
template <> struct Cx<float> { using V = float2; };

inline size_t elem_bytes(diaq_dtype_t t) { return t == DIAQ_C128 ? 16 : 8; }

// Pointers that arrive through memory (the grouped launches' descriptors)
// are generic; casting them to the global address space keeps their
// accesses off the flat path (whose waits would also stall on LDS reads)
// and lets uniform reads use scalar loads.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}

// Native two-element vectors (the element type of interleaved complex
// arrays) for loads and stores through global-space pointers.
template <typename R>
struct Nat;
template <>
struct Nat<double> {
  typedef double T __attribute__((ext_vector_type(2)));
};
template <>
struct Nat<float> {
  typedef float T __attribute__((ext_vector_type(2)));
};

// ---------------------------------------------------------------------------
// Objects behind the opaque handles
// ---------------------------------------------------------------------------

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
  size_t want = 0;  // largest request seen while sizing a graph recording
};

// Recording of a circuit's launches into a HIP graph.  The first recording
// (sizing) is discarded: it only collects the workspace sizes and the bytes
// of host tables; the second runs against workspaces of exactly those sizes
// and stages each table in pinned host memory that the graph copies from on
// every replay.
struct Capture {
  bool sizing = true;
  char* host = nullptr;
  size_t host_bytes = 0;
  size_t host_used = 0;
};

}  // namespace diaq

struct diaq_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 256;
  int lds_bytes = 65536;    // LDS one workgroup may allocate
  diaq::Workspace diag;     // expanded diagonals for circuit runs
  diaq::Workspace red;      // reduction partials
  diaq::Workspace aux;      // small per-call device tables
  double* pinned = nullptr; // host-pinned landing zone for results
  size_t pinned_bytes = 0;
  // SpMV tuning (0 = defaults)
  diaq_tuning_t tuning{};
  int spmv_rows = 0;  // per-call override from a plan
  // kernel timing: events recorded around expansion and product launches
  bool profiling = false;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
  struct Interval {
    size_t ev0, ev1;
    int kind;        // 0 = expansion, 1 = product
    double bytes;
  };
  std::vector<Interval> intervals;
  // set while a circuit graph is being recorded on `stream`
  diaq::Capture* capture = nullptr;
};

struct diaq_dia {
  int32_t nqubits = 0;
  int32_t ndiag = 0;
  diaq_dtype_t dtype = DIAQ_C128;
  std::vector<int64_t> offsets;  // ascending, stored order
  std::vector<int64_t> starts;   // ndiag + 1
  void* values = nullptr;        // device
  int64_t* dmeta = nullptr;      // device: offsets[ndiag] then starts[ndiag+1]
  bool owns_values = false;
  bool transposed = false;       // apply with negated offsets
  bool conjugated = false;       // apply with conjugated values
  uint64_t qubit_mask = 0;       // qubits whose bit the matrix may flip
  bool layout_zeros = false;     // expanded from a gate or a Pauli sum: its zero
                                 // values are structural, the product skips them
  int device = 0;
};

namespace diaq {

// ---------------------------------------------------------------------------
// Host-side gate algebra (gates.cpp)
// ---------------------------------------------------------------------------

struct LocalGate {
  int k = 0;                         // number of targets
  int nc = 0;                        // number of controls
  int targets[3] = {0, 0, 0};
  int controls[3] = {0, 0, 0};
  double m[8][8][2];                 // local matrix, [row][col][re/im]
  bool structural[8][8];             // entry may be non-zero for this kind
  uint64_t tmask = 0, cmask = 0;
};

// Validate a gate against an n-qubit register and build its local matrix.
diaq_status_t local_gate(const diaq_gate_t* g, int n, LocalGate* out);
// Generator G of a rotation kind (U = exp(-i a G / 2)); false if none.
bool local_generator(const diaq_gate_t* g, LocalGate* out);
// Sorted diagonal indices of the expanded gate.
std::vector<int64_t> gate_offsets(const LocalGate& lg);
// Packing starts for offsets of an n-qubit matrix.
std::vector<int64_t> packing_starts(const std::vector<int64_t>& offs, int n);
bool is_diagonal_kind(const diaq_gate_t* g);

// ---------------------------------------------------------------------------
// Gate-level fusion (planner.cpp)
// ---------------------------------------------------------------------------

// A diagonal gate folded into an expansion: the expanded element (i, j) is
// multiplied by v[loc(i)], loc gathering the bits of q[0..k) (q[0] = LSB).
struct DiagFactor {
  int32_t k;
  int32_t q[3];
  double v[8][2];
};

// Device form of an operation's folded diagonal factors.  Diagonal matrices
// commute, so the factors are grouped by qubits and each group's product is
// tabulated once on the host: a table over at most kTableQubits qubits,
// indexed by the element's bits on those qubits.  An element then pays one
// lookup per table instead of one per factor.  Tables follow one another
// in memory: a header, then 2^nq complex entries (16-byte aligned).
constexpr int kTableQubits = 8;
struct TableHead {
  int32_t nq;       // qubits of the table
  int32_t nruns;    // runs of consecutive qubits; none crosses bit 32
  int32_t run[10];  // first qubit | length << 8 | first index bit << 16
  uint8_t roff[32]; // index bits of the operation's row offsets off[r]
};
static_assert(sizeof(TableHead) == 80, "table header is 80 bytes");
inline size_t table_bytes(int nq) { return sizeof(TableHead) + (size_t(16) << nq); }
// Appends the tables of f[0..nf) to *out (planner.cpp); returns how many.
// With row offsets off[0..noff) (noff <= 32; the element offsets of an
// operation's local rows, on bits its cosets leave 0), each header also
// holds roff[r] = the table index bits of off[r].
int compile_factors(const DiagFactor* f, int nf, std::vector<char>* out, const int64_t* off = nullptr,
                    int noff = 0);

// (vr, vi) *= the product of the nt tables at `tabs` at element i.
__device__ __forceinline__ void apply_tables(const char* tabs, int nt, uint64_t i, double& vr, double& vi) {
  // constant address space: the tables are not written while a kernel
  // runs, so the uniform header reads become scalar loads
  typedef __attribute__((address_space(4))) const char GChar;
  typedef __attribute__((address_space(4))) const TableHead GHead;
  typedef __attribute__((address_space(4))) const double GDouble;
  const uint32_t lo = uint32_t(i), hi = uint32_t(i >> 32);
  GChar* p = (GChar*)(tabs);
  for (int t = 0; t < nt; t++) {
    GHead* h = (GHead*)(p);
    const int nq = h->nq, nr = h->nruns;
    uint32_t idx = 0;
    for (int r = 0; r < nr; r++) {
      const uint32_t w = uint32_t(h->run[r]);
      const uint32_t src = w & 63u, len = (w >> 8) & 15u, dst = (w >> 16) & 15u;
      const uint32_t word = src < 32u ? lo : hi;
      idx |= ((word >> (src & 31u)) & ((1u << len) - 1u)) << dst;
    }
    GDouble* e = (GDouble*)(p + sizeof(TableHead));
    const double fr = e[2 * idx], fi = e[2 * idx + 1];
    const double nr2 = vr * fr - vi * fi;
    vi = vr * fi + vi * fr;
    vr = nr2;
    p += sizeof(TableHead) + (size_t(16) << nq);
  }
}

// Rows base | off[r0 + r], r < D, of a coset whose tables were compiled
// with those row offsets: (vr[r], vi[r]) *= the product of the nt tables.
// A table's header is decoded once for all D rows: the coset's index bits
// come from base, each row ORs in the header's roff[r0 + r] (the bit
// gather is linear over disjoint bits).
template <int D>
__device__ __forceinline__ void apply_tables_rows(const char* tabs, int nt, uint64_t base, double (&vr)[D],
                                                  double (&vi)[D], int r0 = 0) {
  typedef __attribute__((address_space(4))) const char GChar;
  typedef __attribute__((address_space(4))) const TableHead GHead;
  typedef __attribute__((address_space(4))) const double GDouble;
  const uint32_t lo = uint32_t(base), hi = uint32_t(base >> 32);
  GChar* p = (GChar*)(tabs);
  for (int t = 0; t < nt; t++) {
    GHead* h = (GHead*)(p);
    const int nq = h->nq, nr = h->nruns;
    uint32_t idx = 0;
    for (int q = 0; q < nr; q++) {
      const uint32_t w = uint32_t(h->run[q]);
      const uint32_t src = w & 63u, len = (w >> 8) & 15u, dst = (w >> 16) & 15u;
      const uint32_t word = src < 32u ? lo : hi;
      idx |= ((word >> (src & 31u)) & ((1u << len) - 1u)) << dst;
    }
    GDouble* e = (GDouble*)(p + sizeof(TableHead));
#pragma unroll
    for (int r = 0; r < D; r++) {
      const uint32_t ir = idx | uint32_t(h->roff[r0 + r]);
      const double fr = e[2 * ir], fi = e[2 * ir + 1];
      const double nr2 = vr[r] * fr - vi[r] * fi;
      vi[r] = vr[r] * fi + vi[r] * fr;
      vr[r] = nr2;
    }
    p += sizeof(TableHead) + (size_t(16) << nq);
  }
}

// Device tables of several operations' factors in one buffer: op k's tables
// start at byte first[k] and number count[k].
struct OpTables {
  std::vector<char> bytes;
  std::vector<size_t> first;
  std::vector<int> count;
  void add(const std::vector<DiagFactor>& post, const int64_t* off = nullptr, int noff = 0) {
    first.push_back(bytes.size());
    count.push_back(post.empty() ? 0 : compile_factors(post.data(), int(post.size()), &bytes, off, noff));
  }
};

// One expansion + product: a core gate (targets, controls, local matrix)
// followed by diagonal gates applied after it.
struct FusedOp {
  LocalGate core;
  std::vector<DiagFactor> post;
  int64_t ngates = 0;  // logical gates folded in
};

// Greedy gate-level fusion: a gate joins the latest op sharing one of its
// qubits (it commutes with every later op) when the product of the local
// matrices (Alg. 1 on the local DiaQ diagonals) spans at most kmax qubits
// and does not move more bytes than the two applied separately; a
// diagonal gate that cannot join the core is folded in as a post factor.
// With kron = true the ops are applied in place by Alg. 3 (2 N s bytes
// each, whatever their diagonals), so any merge within kmax qubits pays.
diaq_status_t plan_fusion(const diaq_gate_t* gates, int64_t ngates, int n, int kmax, diaq_dtype_t dt,
                          std::vector<FusedOp>* ops, bool kron = false);

// Alg. 3 operations of up to five qubits (kronbig.hip): a dense matrix on
// the sorted qubits q (bit j of a local index is q[j]; controls are qubits
// of the group), then diagonal row factors.  A gate of more than five
// qubits with its controls stays raw (its LocalGate).
struct BigOp {
  int k = 0;
  int q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<std::complex<double>> m;
  std::vector<DiagFactor> post;
  uint64_t mask = 0;
  int64_t ngates = 0;
  bool raw = false;
  LocalGate lg;
};
// With kmax = 5 the grouping with a limit of 3, 4 or 5 qubits of least
// modelled time is kept (a dense five-qubit group costs more than a pass
// over the state; dt sets the ratio).
diaq_status_t plan_big(const diaq_gate_t* gates, int64_t ngates, int n, int kmax, std::vector<BigOp>* ops,
                       diaq_dtype_t dt = DIAQ_C128);
// Applies the operations in place (each one read and one write of the
// state), with profiling intervals of 2 s N bytes per operation.
diaq_status_t run_big(diaq_ctx* ctx, const std::vector<BigOp>& ops, int n, diaq_dtype_t dt, void* state);
// An Alg. 3 operation of at most four qubits (targets and controls) that
// touches the lowest qubits runs faster staged through LDS as a dense
// group: true with the dense matrix (interleaved, over the sorted qubits S,
// k of them) if lg qualifies at n qubits (`tables`: it carries factor
// tables).  launch_staged then applies it in place.
bool staged_dense(const LocalGate& lg, int n, int tables, const diaq_tuning_t& t, diaq_dtype_t dt,
                  std::vector<double>* mat, int* S, int* k);
diaq_status_t launch_staged(diaq_ctx* ctx, const int* S, int k, const double* dmat, const char* tabs, int nt, int n,
                            diaq_dtype_t dt, void* state);

// ---------------------------------------------------------------------------
// Kernel launchers (one .hip file each)
// ---------------------------------------------------------------------------

constexpr int kMaxArgDiags = 27;

// Diagonal list passed by value to kernels.
struct DiagArgs {
  int32_t nd;
  int32_t pad;
  int64_t off[kMaxArgDiags];
  int64_t start[kMaxArgDiags];
};

// expand.hip.  `factors` (device, nf entries) are diagonal gates applied
// after the core gate (nullptr / 0: none).
diaq_status_t launch_expand(diaq_ctx* ctx, const LocalGate& lg, int n,
                            diaq_dtype_t dt, const std::vector<int64_t>& offs,
                            const std::vector<int64_t>& starts, void* values,
                            const void* tabs = nullptr, int nt = 0);
diaq_status_t launch_pauli_dia(diaq_ctx* ctx, int n, diaq_dtype_t dt,
                               const std::vector<int64_t>& offs,
                               const std::vector<int64_t>& starts,
                               const uint64_t* xm, const uint64_t* zm,
                               const double* coef, int nterms, void* values);

// spmv.hip.  The matrix is (offsets, starts, values) with optional
// transpose / conjugation; offsets come from `args` when nd <= kMaxArgDiags,
// else from the device table dmeta.
struct SpmvOp {
  int n = 0;
  diaq_dtype_t dtype = DIAQ_C128;
  int nd = 0;
  const int64_t* host_off = nullptr;    // host view (for planning)
  const int64_t* host_start = nullptr;
  const int64_t* dmeta = nullptr;       // device table (nd > kMaxArgDiags)
  const void* values = nullptr;
  bool transpose = false;
  bool conjugate = false;
  uint64_t qubit_mask = 0;
  // the matrix was expanded from a gate or a Pauli sum: its exact zeros are
  // structural and their x loads are skipped; otherwise every stored
  // element multiplies its x entry (a non-finite x propagates, as in Alg. 2)
  bool skip_zero = false;
};
diaq_status_t launch_spmv(diaq_ctx* ctx, const SpmvOp& op, const void* x,
                          void* y);
// The launch shape launch_spmv would choose for op under the knobs t.
diaq_status_t spmv_shape(const SpmvOp& op, const diaq_tuning_t& t, diaq_spmv_shape_t* out);

// expect.hip: out2 = <psi | op | phi> reduced deterministically; result left
// in device memory at dres (2 doubles).
diaq_status_t launch_expect(diaq_ctx* ctx, const SpmvOp& op, const void* psi,
                            const void* phi, double* dres);
// The same product and reduction with its partial sums in the library's
// static device array (kStaticPartials entries per device) instead of a
// context workspace: allocates nothing; products that need more partials
// return DIAQ_ERR_UNSUPPORTED.  init_static_scratch(device), called with
// that device current (diaq_create), takes the array's device address.
constexpr int64_t kStaticPartials = int64_t(1) << 20;
constexpr int kMaxStaticDevices = 64;
diaq_status_t init_static_scratch(int device);
diaq_status_t launch_expect_static(diaq_ctx* ctx, const SpmvOp& op, const void* psi,
                                   const void* phi, double* dres);
// <lam | G | psi> for a local generator applied by index bit manipulation.
diaq_status_t launch_generator_dot(diaq_ctx* ctx, const LocalGate& gen, int n,
                                   diaq_dtype_t dt, const void* lam,
                                   const void* psi, double* dres);

// kron.hip: Alg. 3 products without expansion, in place on `v`.  `dmat`
// (device, 4 x 4 complex, at most 2 targets) replaces lg's matrix when the
// matrix depends on angles that live on the device.
// `rows`: the tables were compiled with the row offsets kron_row_offsets
// gives for lg (one header decode per coset instead of one per row).
diaq_status_t launch_kron_apply(diaq_ctx* ctx, hipStream_t stream, const LocalGate& lg, int n, diaq_dtype_t dt,
                                void* v, bool adjoint, const void* tabs = nullptr, int nt = 0,
                                const double* dmat = nullptr, bool rows = false);
// off[r] (r < 2^lg.k): the element offset of local row r (bit j of r on
// qubit lg.targets[j]), as the Alg. 3 kernels address a coset's rows.
void kron_row_offsets(const LocalGate& lg, int64_t* off);
// Reverse-sweep step: optional generator dot (one double2 partial per
// workgroup into `partial`, kron_adjoint_blocks of them), then
// psi, lam <- U^dagger psi, U^dagger lam when step_back.
int64_t kron_adjoint_blocks(const LocalGate& lg, int n);
diaq_status_t launch_kron_adjoint(diaq_ctx* ctx, hipStream_t stream, const LocalGate& lg, const LocalGate* gen,
                                  int n, diaq_dtype_t dt, void* psi, void* lam, double2* partial, bool step_back,
                                  const double* dmat = nullptr);
// small.hip: the gates lg applied in order to a state small enough for
// one workgroup's LDS (one launch per run of gates that fits the kernel
// arguments), in place.
diaq_status_t run_small(diaq_ctx* ctx, const std::vector<LocalGate>& lg, int n, diaq_dtype_t dt, void* state);
// Largest register the one-launch path takes for the knobs and the device.
int small_circuit_qubits(const diaq_ctx* ctx, diaq_dtype_t dt);
// spmv.hip: one workgroup sums partial[0..count) into dres (2 doubles).
// Algorithmic bytes of one Alg. 3 operation: every amplitude it changes is
// read and written once.  Without folded factors only the rows whose
// controls are all 1 change (1 / 2^nc of the state); folded factors touch
// every row.
double kron_op_bytes(const LocalGate& core, int nf, int n, diaq_dtype_t dt);
// ---------------------------------------------------------------------------
// Segmented adjoint sweep (segment.hip)
// ---------------------------------------------------------------------------

// One gate of a segment in the coset's local basis (bit j of a local index
// is qubit S[j], S ascending).
struct SegGate {
  int32_t kind;     // 0: one target, 1: two targets, 2: three targets (= S), 3: diagonal,
                    // 4: header of a run of b0 diagonal phase gates, 5: member of a run
  int32_t b0, b1;   // local bits of targets 0 and 1 (kinds 0, 1)
  int32_t dot;      // slot of this gate's dot within the segment, -1 if none
  int32_t dk;       // diagonal: number of qubits in q
  int32_t q[3];     // diagonal: the gate's qubits, q[0] = bit 0 of its table
  uint64_t cmask;   // controls: the gate acts where all are 1
  int64_t moff;     // doubles into the pool: U^dagger, then the generator
};

struct Segment {
  int S[3];            // coset qubits, ascending
  int64_t first = 0;   // first SegGate
  int64_t ngates = 0;
  int32_t ndots = 0;
  int64_t dot_slot0 = 0;  // first entry of SegmentPlan::dot_gate
  bool three = false;     // holds a three-target gate
  int64_t pool_lo = 0, pool_n = 0;  // its matrices in SegmentPlan::pool
};

struct SegmentPlan {
  bool forward = false;          // circuit order with U (no dots) instead of the reverse sweep
  std::vector<SegGate> gates;    // all segments, each in sweep order
  std::vector<int64_t> gate_of;  // circuit gate index of each SegGate
  std::vector<double> pool;      // matrices
  std::vector<Segment> segs;     // in sweep order (last gates first)
  std::vector<int64_t> dot_gate; // circuit gate index of each dot, by segment
};

constexpr int kSegMaxDots = 64;
constexpr int kSegLdsGates = 128;   // SegGate entries of one segment
constexpr int kSegLdsPool = 2048;   // matrix doubles of one segment (its diagonal tables are staged in LDS)

// Cut the reverse sweep (or, with forward, the circuit in its own order)
// into segments: consecutive gates whose non-diagonal targets fit in 3
// qubits (diagonal gates and controls anywhere).  dkey[g] >= 0 marks gates
// whose dot the reverse sweep takes (gens[g] is then their generator);
// consecutive diagonal gates with equal keys (same parameter and scale)
// share one dot, stored at the first of them (SegmentPlan::dot_gate).
diaq_status_t plan_segments(const std::vector<LocalGate>& lg, const std::vector<LocalGate>& gens,
                            const std::vector<int64_t>& dkey, int n, SegmentPlan* out, bool forward = false);
// Device table layout [gates | pool | dot output slots]: its size, and its
// host image with slots[j] = output slot (pairs of doubles) of dot j.
size_t segment_table_bytes(const SegmentPlan& P);
void segment_table_host(const SegmentPlan& P, std::vector<char>& host, const std::vector<int64_t>& slots);
// The reverse sweep's partial sums: every segment has its own rows (this
// many double2 entries in all), and the table's last region holds one
// reduce record per segment with dots, filled in by segment_table_reds
// once the device addresses of the table and of the partials are known.
int64_t segment_partial_entries(const SegmentPlan& P, int n);
size_t segment_reds_offset(const SegmentPlan& P);
void segment_table_reds(const SegmentPlan& P, int n, const void* table_dev, const double2* partial,
                        std::vector<char>& host);
int64_t segment_blocks(int n);
// Byte offset of the matrix pool inside the device table.
size_t segment_pool_offset(const SegmentPlan& P);

// Grouped sweeps over many independent complex128 states: step k runs
// segment k of every item's plan in one launch (workgroups of the items one
// after another), then, for reverse plans, all of that step's dot sums in a
// second launch.  The descriptors hold device pointers only; `host` is
// their image, to be copied to `dev` (G.host.size() bytes) before running.
struct GroupItem {
  const SegmentPlan* plan;
  const void* table;     // device table of the plan
  int n;
  void* psi;
  void* lam;             // reverse plans
  double2* partial;      // reverse plans: segment_blocks(n) * (max dots of a segment) entries
};
struct GroupedStep {
  int64_t seg_first = 0, seg_count = 0, blocks = 0;
  int64_t red_first = 0, red_count = 0, red_blocks = 0;
  bool three = false;
};
struct GroupedSweep {
  bool forward = false;
  std::vector<GroupedStep> steps;
  std::vector<char> host;
  size_t red_offset = 0;
  const void* dev = nullptr;
};
diaq_status_t build_grouped(const std::vector<GroupItem>& items, bool forward, GroupedSweep* out);
diaq_status_t run_grouped(hipStream_t stream, const GroupedSweep& G, double* dots);
// Run the sweep: for every segment one pass over psi and lambda (each dot
// taken before its gate is undone), then the fixed-order dot sums into
// dots[2 * slot], dots[2 * slot + 1].  partial holds segment_blocks(n) *
// kSegMaxDots entries.  A forward plan passes over psi alone (lam,
// partial and dots unused).
diaq_status_t run_segments(diaq_ctx* ctx, hipStream_t stream, const SegmentPlan& P, int n, diaq_dtype_t dt,
                           void* psi, void* lam, void* table_mem, double2* partial, double* dots);

diaq_status_t launch_final_reduce(hipStream_t stream, const double2* partial, int64_t count, double* dres);

// fuse.hip
diaq_status_t fuse_dia(diaq_ctx* ctx, const diaq_dia* first,
                       const diaq_dia* second, double drop_tol,
                       diaq_dia** out);

// Workspace growth (never shrinks).
diaq_status_t ensure(diaq_ctx* ctx, Workspace* w, size_t bytes);
// Device-to-device copy by a streaming kernel (16-byte aligned, a multiple
// of 16 bytes, no overlap).
diaq_status_t launch_copy(hipStream_t stream, const void* src, void* dst, size_t bytes);
// dst <- 0 by a kernel (16-byte aligned, a multiple of 16 bytes).
diaq_status_t launch_zero(hipStream_t stream, void* dst, size_t bytes);
// Copy a host table that dies with the calling function into device memory
// ahead of the launches that read it: synchronous (after the stream's
// earlier work) when running eagerly, a copy node from pinned staging when
// a graph is being recorded.
diaq_status_t upload(diaq_ctx* ctx, void* dst, const void* src, size_t bytes);
diaq_status_t ensure_pinned(diaq_ctx* ctx, size_t bytes);

// Qubit mask of the off-diagonal structure implied by an offset list.
uint64_t mask_from_offsets(const std::vector<int64_t>& offs);

diaq_status_t new_dia(diaq_ctx* ctx, int n, diaq_dtype_t dt,
                      const std::vector<int64_t>& offs, void* values,
                      bool zero_fill, diaq_dia** out);

// SpMV operand view of a DiaQ matrix with the given effective flags.
SpmvOp op_of(const diaq_dia* A, bool transpose, bool conjugate);

// Kernel timing: record an event on the context stream (returns its index
// in ctx->events, or SIZE_MAX when profiling is off) and close an interval.
size_t prof_mark(diaq_ctx* ctx);
void prof_interval(diaq_ctx* ctx, size_t ev0, size_t ev1, int kind, double bytes);

}  // namespace diaq

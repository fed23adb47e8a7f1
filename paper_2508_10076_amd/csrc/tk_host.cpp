// Host side of the symmetric-TensorMap library: graded spaces, block
// structure of TensorMaps, permute and contraction plans, tile scheduling,
// plan cache and the C-ABI declared in include/tk.h.  Only planning happens
// here; every numerical step runs in the kernels of tk_kernels.hip.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <queue>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "tk.h"
#include "tk_internal.h"

using tk::GemmDesc;
using tk::GemmTile;
using tk::LegMap;
using tk::PairDesc;
using tk::PermTask;

namespace {

thread_local std::string g_err;

struct TkError {
  tk_status st;
  std::string msg;
};

[[noreturn]] void fail(tk_status st, const std::string& msg) { throw TkError{st, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(TK_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// symmetries and spaces
// ---------------------------------------------------------------------------
struct SymInfo {
  int ncomp;
  bool has_q, has_p, fermionic;
};

SymInfo sym_info(int sym) {
  switch (sym) {
    case TK_SYM_Z1: return {0, false, false, false};
    case TK_SYM_Z2: return {1, false, true, false};
    case TK_SYM_FZ2: return {1, false, true, true};
    case TK_SYM_U1: return {1, true, false, false};
    case TK_SYM_U1_FZ2: return {2, true, true, true};
    default: fail(TK_ERR_INVALID_ARG, "unknown symmetry " + std::to_string(sym));
  }
}

// A graded space: sectors (U(1) charge q, parity p; unused components are 0),
// degeneracies, dual flag.  The label of sector k on this leg is the sector
// itself on a normal space and its conjugate (-q, p) on a dual space.
struct Space {
  std::vector<int32_t> q, p;
  std::vector<int64_t> deg;
  bool dual = false;
  std::vector<int32_t> raw;  // charges as given (nsect * ncomp), for tk_tensor_space

  int n() const { return static_cast<int>(deg.size()); }
  int64_t lab_q(int k) const { return dual ? -static_cast<int64_t>(q[k]) : q[k]; }
  Space flipped() const {
    Space s = *this;
    s.dual = !dual;
    return s;
  }
  bool operator==(const Space& o) const { return q == o.q && p == o.p && deg == o.deg && dual == o.dual; }
  bool operator!=(const Space& o) const { return !(*this == o); }
};

inline int64_t make_key(int64_t q, int p) { return 2 * q + p; }

Space make_space(int sym, const tk_space& s) {
  SymInfo si = sym_info(sym);
  if (s.nsect < 1 || s.nsect > 255) fail(TK_ERR_UNSUPPORTED, "a space needs 1..255 sectors");
  if (!s.degeneracies) fail(TK_ERR_INVALID_ARG, "null degeneracies");
  if (si.ncomp > 0 && !s.charges) fail(TK_ERR_INVALID_ARG, "null charges");
  if (sym == TK_SYM_Z1 && s.nsect != 1) fail(TK_ERR_CHARGE, "Z1 spaces have exactly one sector");
  Space sp;
  sp.dual = s.isdual != 0;
  for (int k = 0; k < s.nsect; ++k) {
    int32_t q = 0, p = 0;
    if (sym == TK_SYM_Z2 || sym == TK_SYM_FZ2) p = s.charges[k];
    if (sym == TK_SYM_U1) q = s.charges[k];
    if (sym == TK_SYM_U1_FZ2) {
      q = s.charges[2 * k];
      p = s.charges[2 * k + 1];
    }
    if (si.has_p && (p < 0 || p > 1)) fail(TK_ERR_CHARGE, "parity must be 0 or 1");
    if (si.has_q && (q < -(1 << 24) || q > (1 << 24))) fail(TK_ERR_CHARGE, "charge out of range");
    if (s.degeneracies[k] < 1 || s.degeneracies[k] > (int64_t(1) << 31) - 1)
      fail(TK_ERR_INVALID_ARG, "degeneracies must be in 1 .. 2^31-1");
    for (int j = 0; j < k; ++j)
      if (sp.q[j] == q && sp.p[j] == p) fail(TK_ERR_CHARGE, "repeated sector in a space");
    sp.q.push_back(q);
    sp.p.push_back(p);
    sp.deg.push_back(s.degeneracies[k]);
    for (int c = 0; c < si.ncomp; ++c) sp.raw.push_back(s.charges[si.ncomp * k + c]);
  }
  return sp;
}

// ---------------------------------------------------------------------------
// block structure
// ---------------------------------------------------------------------------
// Channels of one side with one coupled label, in colexicographic order
// (first leg fastest).  off is the row (column) offset inside t^(c).
struct Group {
  std::vector<uint8_t> idx;  // n * nlegs sector indices
  std::vector<int64_t> size, off;
  int64_t total = 0;
  int32_t n() const { return static_cast<int32_t>(size.size()); }
};

struct Side {
  int nlegs = 0;
  std::map<int64_t, Group> groups;
  mutable std::mutex mu;
  mutable std::unordered_map<uint64_t, int32_t> lookup;  // packed tuple -> index in its group
  mutable bool lookup_built = false;

  static uint64_t pack(const uint8_t* t, int n) {
    uint64_t k = 0;
    for (int l = 0; l < n; ++l) k |= static_cast<uint64_t>(t[l]) << (8 * l);
    return k;
  }
  int32_t find(const uint8_t* t) const {
    std::lock_guard<std::mutex> g(mu);
    if (!lookup_built) {
      for (const auto& kv : groups) {
        const Group& gr = kv.second;
        for (int32_t i = 0; i < gr.n(); ++i) lookup[pack(gr.idx.data() + size_t(i) * nlegs, nlegs)] = i;
      }
      lookup_built = true;
    }
    auto it = lookup.find(pack(t, nlegs));
    return it == lookup.end() ? -1 : it->second;
  }
};

struct Structure {
  int sym = 0;
  SymInfo si{};
  std::vector<Space> cod, dom;
  Side rows, cols;
  std::vector<int64_t> keys;  // coupled labels present on both sides, ascending
  std::vector<const Group*> rg, cg;
  std::vector<int64_t> R, C, soff, bbase;
  int64_t size = 0, nblocks = 0;
  std::string sig;

  int N1() const { return static_cast<int>(cod.size()); }
  int N2() const { return static_cast<int>(dom.size()); }
  int N() const { return N1() + N2(); }
  const Space& leg(int l) const { return l < N1() ? cod[l] : dom[l - N1()]; }
  int sector_of_key(int64_t key) const {
    auto it = std::lower_bound(keys.begin(), keys.end(), key);
    return (it != keys.end() && *it == key) ? static_cast<int>(it - keys.begin()) : -1;
  }
  int64_t tuple_key(const std::vector<Space>& legs, const uint8_t* t) const {
    int64_t q = 0;
    int p = 0;
    for (size_t l = 0; l < legs.size(); ++l) {
      q += legs[l].lab_q(t[l]);
      p ^= legs[l].p[t[l]];
    }
    return make_key(q, p);
  }
};

void enumerate_side(const std::vector<Space>& legs, const std::vector<int64_t>* keep, Side& out) {
  const int N = static_cast<int>(legs.size());
  out.nlegs = N;
  if (N == 0) {
    if (!keep || std::binary_search(keep->begin(), keep->end(), make_key(0, 0))) {
      Group g;
      g.size = {1};
      g.off = {0};
      g.total = 1;
      out.groups[make_key(0, 0)] = std::move(g);
    }
    return;
  }
  int64_t qmin = 0, qmax = 0;
  for (const auto& s : legs) {
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int k = 0; k < s.n(); ++k) {
      lo = std::min(lo, s.lab_q(k));
      hi = std::max(hi, s.lab_q(k));
    }
    qmin += lo;
    qmax += hi;
  }
  const int64_t kmin = make_key(qmin, 0), nkeys = make_key(qmax, 1) - kmin + 1;
  std::vector<Group> flat;
  std::map<int64_t, Group> sparse;
  const bool use_flat = nkeys <= (1 << 20);
  if (use_flat) flat.resize(static_cast<size_t>(nkeys));
  std::vector<char> keep_flat;
  if (keep && use_flat) {
    keep_flat.assign(static_cast<size_t>(nkeys), 0);
    for (int64_t k : *keep)
      if (k >= kmin && k < kmin + nkeys) keep_flat[static_cast<size_t>(k - kmin)] = 1;
  }
  // odometer over legs 1..N-1, inner loop over leg 0 (first leg fastest)
  std::vector<int> cur(N, 0);
  std::vector<uint8_t> tup(N, 0);
  while (true) {
    int64_t q = 0, sz = 1;
    int p = 0;
    for (int l = 1; l < N; ++l) {
      q += legs[l].lab_q(cur[l]);
      p ^= legs[l].p[cur[l]];
      sz *= legs[l].deg[cur[l]];
      tup[l] = static_cast<uint8_t>(cur[l]);
    }
    const Space& l0 = legs[0];
    for (int k = 0; k < l0.n(); ++k) {
      const int64_t key = make_key(q + l0.lab_q(k), p ^ l0.p[k]);
      Group* g;
      if (use_flat) {
        if (keep && !keep_flat[static_cast<size_t>(key - kmin)]) continue;
        g = &flat[static_cast<size_t>(key - kmin)];
      } else {
        if (keep && !std::binary_search(keep->begin(), keep->end(), key)) continue;
        g = &sparse[key];
      }
      tup[0] = static_cast<uint8_t>(k);
      const int64_t s = sz * l0.deg[k];
      g->idx.insert(g->idx.end(), tup.begin(), tup.end());
      g->off.push_back(g->total);
      g->size.push_back(s);
      g->total += s;
    }
    int l = 1;
    while (l < N) {
      if (++cur[l] < legs[l].n()) break;
      cur[l] = 0;
      ++l;
    }
    if (l >= N) break;
  }
  if (use_flat) {
    for (int64_t i = 0; i < nkeys; ++i)
      if (!flat[static_cast<size_t>(i)].size.empty()) out.groups[kmin + i] = std::move(flat[static_cast<size_t>(i)]);
  } else {
    out.groups = std::move(sparse);
  }
}

std::string space_sig(const Space& s) {
  std::string r = s.dual ? "D" : "N";
  for (int k = 0; k < s.n(); ++k)
    r += std::to_string(s.q[k]) + "," + std::to_string(s.p[k]) + ":" + std::to_string(s.deg[k]) + ";";
  return r;
}

std::string structure_sig(int sym, const std::vector<Space>& cod, const std::vector<Space>& dom) {
  std::string r = "S" + std::to_string(sym) + "|";
  for (const auto& s : cod) r += space_sig(s) + "|";
  r += "->|";
  for (const auto& s : dom) r += space_sig(s) + "|";
  return r;
}

std::shared_ptr<Structure> build_structure(int sym, const std::vector<Space>& cod, const std::vector<Space>& dom) {
  if (cod.size() > TK_MAX_LEGS || dom.size() > TK_MAX_LEGS || cod.size() + dom.size() > TK_MAX_RANK)
    fail(TK_ERR_UNSUPPORTED, "too many legs");
  auto st = std::make_shared<Structure>();
  st->sym = sym;
  st->si = sym_info(sym);
  st->cod = cod;
  st->dom = dom;
  st->sig = structure_sig(sym, cod, dom);
  // enumerate the smaller side first and keep only its labels on the other
  auto side_count = [](const std::vector<Space>& v) {
    double c = 1;
    for (const auto& s : v) c *= s.n();
    return c;
  };
  std::vector<int64_t> keys;
  if (side_count(dom) <= side_count(cod)) {
    enumerate_side(dom, nullptr, st->cols);
    for (const auto& kv : st->cols.groups) keys.push_back(kv.first);
    enumerate_side(cod, &keys, st->rows);
  } else {
    enumerate_side(cod, nullptr, st->rows);
    for (const auto& kv : st->rows.groups) keys.push_back(kv.first);
    enumerate_side(dom, &keys, st->cols);
  }
  int64_t off = 0, nb = 0;
  for (const auto& kv : st->rows.groups) {
    auto it = st->cols.groups.find(kv.first);
    if (it == st->cols.groups.end()) continue;
    st->keys.push_back(kv.first);
    st->rg.push_back(&kv.second);
    st->cg.push_back(&it->second);
    st->R.push_back(kv.second.total);
    st->C.push_back(it->second.total);
    st->soff.push_back(off);
    st->bbase.push_back(nb);
    off += kv.second.total * it->second.total;
    nb += static_cast<int64_t>(kv.second.n()) * it->second.n();
  }
  st->size = off;
  st->nblocks = nb;
  return st;
}

std::mutex g_struct_mu;
std::unordered_map<std::string, std::weak_ptr<Structure>> g_struct_cache;

std::shared_ptr<Structure> get_structure(int sym, const std::vector<Space>& cod, const std::vector<Space>& dom) {
  const std::string sig = structure_sig(sym, cod, dom);
  {
    std::lock_guard<std::mutex> g(g_struct_mu);
    auto it = g_struct_cache.find(sig);
    if (it != g_struct_cache.end())
      if (auto sp = it->second.lock()) return sp;
  }
  auto st = build_structure(sym, cod, dom);
  std::lock_guard<std::mutex> g(g_struct_mu);
  g_struct_cache[sig] = st;
  return st;
}

// Space assignment of Alg. "Tensor Permute": V'_i = p_i-th of (V.., W*..),
// W'_j = q_j-th of (V*.., W..).
void permute_spaces(const Structure& A, const std::vector<int>& p, const std::vector<int>& q,
                    std::vector<Space>& cod, std::vector<Space>& dom) {
  cod.clear();
  dom.clear();
  for (int i : p) cod.push_back(i < A.N1() ? A.leg(i) : A.leg(i).flipped());
  for (int j : q) dom.push_back(j < A.N1() ? A.leg(j).flipped() : A.leg(j));
}

std::vector<int> to_vec(const int32_t* a, int32_t n, const char* what) {
  if (n < 0 || (n > 0 && !a)) fail(TK_ERR_INVALID_ARG, std::string("bad index list ") + what);
  return std::vector<int>(a, a + n);
}

void check_perm(const std::vector<int>& p, const std::vector<int>& q, int N) {
  if (static_cast<int>(p.size() + q.size()) != N) fail(TK_ERR_INVALID_ARG, "(p, q) must list every leg once");
  std::vector<char> seen(N, 0);
  for (int v : p) {
    if (v < 0 || v >= N || seen[v]) fail(TK_ERR_INVALID_ARG, "(p, q) is not a permutation of the legs");
    seen[v] = 1;
  }
  for (int v : q) {
    if (v < 0 || v >= N || seen[v]) fail(TK_ERR_INVALID_ARG, "(p, q) is not a permutation of the legs");
    seen[v] = 1;
  }
  if (p.size() > TK_MAX_LEGS || q.size() > TK_MAX_LEGS) fail(TK_ERR_UNSUPPORTED, "too many legs on one side");
}

bool is_identity(const std::vector<int>& p, const std::vector<int>& q, int N1) {
  if (static_cast<int>(p.size()) != N1) return false;
  for (size_t i = 0; i < p.size(); ++i)
    if (p[i] != static_cast<int>(i)) return false;
  for (size_t j = 0; j < q.size(); ++j)
    if (q[j] != static_cast<int>(N1 + j)) return false;
  return true;
}

// Exchanged leg pairs of a permutation: pairs of input legs (x, y) whose
// order in the bra-ket reading (codomain, then domain reversed) flips.
std::vector<std::pair<int, int>> exchanged_pairs(int N1, int N2, const std::vector<int>& p, const std::vector<int>& q) {
  const int N = N1 + N2;
  std::vector<int> pos_in(N), pos_out(N);
  for (int l = 0; l < N1; ++l) pos_in[l] = l;
  for (int j = 0; j < N2; ++j) pos_in[N1 + j] = N - 1 - j;
  const int n1o = static_cast<int>(p.size());
  for (int i = 0; i < n1o; ++i) pos_out[p[i]] = i;
  for (size_t j = 0; j < q.size(); ++j) pos_out[q[j]] = N - 1 - static_cast<int>(j);
  std::vector<std::pair<int, int>> r;
  for (int x = 0; x < N; ++x)
    for (int y = 0; y < N; ++y)
      if (pos_in[x] < pos_in[y] && pos_out[x] > pos_out[y]) r.emplace_back(x, y);
  return r;
}

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
static_assert(TK_SCRATCH_BYTES == tk::kScratchBytes, "scratch size of tk.h and the kernels differ");

struct DevBuf;

// Device allocations the library has made (tk_device_alloc_count).
std::atomic<uint64_t> g_device_allocs{0};

// Placement of one allocation-free call's device memory.  While an arena is
// active on the calling thread, DevBuf::alloc and DevBuf::upload record
// requests instead of allocating: uploaded tables are staged back to back
// (256-byte aligned) in host memory, workspaces only reserve their size.
// place() then gives every request an address inside the caller's region
// (tables first, then workspaces) and copies the staged tables in with one
// asynchronous host-to-device copy.
struct Arena {
  struct Req {
    DevBuf* buf;
    size_t off, bytes;
    bool table;
  };
  std::vector<Req> reqs;
  std::vector<char>* staging = nullptr;  // table bytes (owned by the caller)
  size_t work = 0;                       // workspace bytes reserved so far
  static size_t align(size_t x) { return (x + 255) & ~size_t(255); }
  void reserve(DevBuf* b, size_t n) {
    reqs.push_back({b, work, n, false});
    work += align(n);
  }
  void stage(DevBuf* b, const void* src, size_t n) {
    const size_t off = staging->size();
    staging->resize(align(off + n));
    std::memcpy(staging->data() + off, src, n);
    reqs.push_back({b, off, n, true});
  }
  size_t total() const { return staging->size() + work; }
  void place(char* base, size_t cap, hipStream_t stream);
};
thread_local Arena* t_arena = nullptr;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool borrowed = false;  // p lies in an arena's region (never freed here)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && !borrowed) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    borrowed = false;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    if (t_arena) {
      t_arena->reserve(this, n);
      return;
    }
    if (hipMalloc(&p, n) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      fail(TK_ERR_OOM, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    g_device_allocs.fetch_add(1, std::memory_order_relaxed);
    bytes = n;
  }
  template <typename T>
  void upload(const std::vector<T>& v) {
    if (t_arena) {
      release();
      if (!v.empty()) t_arena->stage(this, v.data(), v.size() * sizeof(T));
      return;
    }
    alloc(v.size() * sizeof(T));
    if (!v.empty()) hip_check(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  }
};

void Arena::place(char* base, size_t cap, hipStream_t stream) {
  const size_t tab = staging->size();
  if (total() > cap)
    fail(TK_ERR_UNSUPPORTED, "the contraction needs " + std::to_string(total()) +
                                 " bytes of scratch (tables and workspaces); the allocation-free entry point has " +
                                 std::to_string(cap));
  for (const Req& r : reqs) {
    r.buf->p = base + (r.table ? r.off : tab + r.off);
    r.buf->bytes = r.bytes;
    r.buf->borrowed = true;
  }
  if (tab) hip_check(hipMemcpyAsync(base, staging->data(), tab, hipMemcpyHostToDevice, stream), "scratch table copy");
}

// ---------------------------------------------------------------------------
// permute task lists
// ---------------------------------------------------------------------------
template <typename TaskT>
struct TaskListT {
  std::vector<TaskT> tasks;
  std::vector<int32_t> wg_first{0};
  std::vector<tk::TileTask> tiles;  // LDS-staged tiles (block permutes only)
  DevBuf d_tasks, d_wg, d_tiles;
  int nwg() const { return static_cast<int>(wg_first.size()) - 1; }
  int ntiles() const { return static_cast<int>(tiles.size()); }
  void upload() {
    d_tasks.upload(tasks);
    d_wg.upload(wg_first);
    d_tiles.upload(tiles);
  }
};

using TaskList = TaskListT<PermTask>;

// Enqueue a permute task list: the output-order walk over its tasks, then
// its LDS-staged tiles.
void launch_tasklist(int dtype, const TaskList& tl, const tk::Ptrs& ptrs, double alpha, double beta,
                     hipStream_t stream, bool split, const char* what) {
  if (tl.nwg() > 0)
    hip_check(tk::launch_permute(dtype, static_cast<const PermTask*>(tl.d_tasks.p),
                                 static_cast<const int32_t*>(tl.d_wg.p), tl.nwg(), ptrs, alpha, beta, stream, split),
              what);
  if (tl.ntiles() > 0)
    hip_check(tk::launch_permute_tiles(dtype, static_cast<const tk::TileTask*>(tl.d_tiles.p), tl.ntiles(), ptrs,
                                       alpha, beta, stream, split),
              what);
}
using SkBlockList = TaskListT<tk::SkBlockTask>;

// Limits of the workgroup tables of the zero-range and output-run kernels,
// which stage a workgroup's items in LDS arrays of max_items + 1 entries and
// index its elements (at most chunk) through an LDS map: every item holds at
// least one element, workgroup w covers elements wstart[w] .. wstart[w+1]-1
// (1..chunk of them), item first[w] holds its first element, first[] never
// decreases, and the items from first[w] to first[w+1] (the last one may
// start exactly at the workgroup's end) number at most max_items + 1.  A
// violation is a planner bug; it fails the plan instead of reaching a kernel.
void check_chunks(const std::vector<int64_t>& vstart, int64_t total, const std::vector<int32_t>& first,
                  const std::vector<int64_t>& wstart, int chunk, int max_items, const char* what) {
  const int64_t n = static_cast<int64_t>(vstart.size());
  auto bad = [&](const char* why) { fail(TK_ERR_UNSUPPORTED, std::string(what) + " work list: " + why); };
  for (int64_t i = 0; i < n; ++i) {
    const int64_t end = i + 1 < n ? vstart[i + 1] : total;
    if (end - vstart[i] < 1) bad("an item without elements");
  }
  if (n == 0) return;
  if (first.size() != wstart.size() || wstart.size() < 2 || wstart.front() != 0 || wstart.back() != total)
    bad("workgroup bounds");
  for (size_t w = 0; w + 1 < wstart.size(); ++w) {
    const int64_t len = wstart[w + 1] - wstart[w];
    if (len < 1 || len > chunk) bad("workgroup size");
    const int32_t f = first[w], f1 = first[w + 1];
    if (f < 0 || f1 < f || f1 >= n) bad("item order");
    const int64_t fend = f + 1 < n ? vstart[f + 1] : total;
    if (vstart[f] > wstart[w] || fend <= wstart[w]) bad("first item does not hold the first element");
    if (static_cast<int64_t>(std::min<int64_t>(n, static_cast<int64_t>(f1) + 1)) - f > max_items + 1)
      bad("too many items in one workgroup");
  }
}

// Ranges of elements to zero: collected as (buffer, offset, length), then
// sorted, merged where adjacent, and laid end to end as one virtual array
// cut into workgroups of at most kZeroChunk elements in at most kZeroMax
// ranges.
struct ZeroSet {
  std::vector<std::tuple<int32_t, int64_t, int64_t>> raw;
  std::vector<tk::ZeroRange> ranges;
  std::vector<int32_t> first;
  std::vector<int64_t> wstart;
  int64_t total = 0;
  DevBuf d_ranges, d_first, d_wstart;
  void add(int32_t buf, int64_t off, int64_t len) {
    if (len > 0) raw.emplace_back(buf, off, len);
  }
  void finalize() {
    std::sort(raw.begin(), raw.end());
    ranges.clear();
    total = 0;
    int64_t end = -1;
    int32_t cur = -1;
    for (const auto& r : raw) {
      const int32_t buf = std::get<0>(r);
      const int64_t off = std::get<1>(r), len = std::get<2>(r);
      if (!(buf == cur && off == end)) {
        tk::ZeroRange z{};
        z.off = off;
        z.vstart = total;
        z.buf = buf;
        ranges.push_back(z);
      }
      cur = buf;
      end = off + len;
      total += len;
    }
    if (ranges.size() > static_cast<size_t>(INT32_MAX)) fail(TK_ERR_UNSUPPORTED, "too many zero ranges");
    first.clear();
    wstart.clear();
    if (ranges.empty()) return;
    int64_t v = 0;
    size_t r = 0;
    wstart.push_back(0);
    first.push_back(0);
    while (v < total) {
      int64_t stop = std::min(total, v + tk::kZeroChunk);
      if (r + tk::kZeroMax < ranges.size()) stop = std::min(stop, ranges[r + tk::kZeroMax].vstart);
      v = stop;
      while (r + 1 < ranges.size() && ranges[r + 1].vstart <= v) ++r;
      wstart.push_back(v);
      first.push_back(static_cast<int32_t>(r));
    }
    if (wstart.size() - 1 > static_cast<size_t>(INT32_MAX)) fail(TK_ERR_UNSUPPORTED, "zero fill too large");
    std::vector<int64_t> vs(ranges.size());
    for (size_t i = 0; i < ranges.size(); ++i) vs[i] = ranges[i].vstart;
    check_chunks(vs, total, first, wstart, tk::kZeroChunk, tk::kZeroMax, "zero-range");
  }
  int nwg() const { return wstart.empty() ? 0 : static_cast<int>(wstart.size()) - 1; }
  void upload() {
    d_ranges.upload(ranges);
    d_first.upload(first);
    d_wstart.upload(wstart);
  }
};

// bound of the output-run decoder's 24-bit arithmetic
constexpr int64_t kRunLimit = int64_t(1) << 24;

// Output runs and block decoders of the small-K sectors of one K value.
// Workgroups cut the concatenation of the runs (in destination order) into
// pieces of at most kRunChunk elements touching at most kRunMax runs.
struct RunSet {
  std::vector<tk::SkRun> runs;
  std::vector<tk::SkRunShape> shapes;
  std::map<std::string, int32_t> shape_id;  // shape bytes -> index
  std::vector<int32_t> first;
  std::vector<int64_t> wstart;
  int64_t total = 0;
  DevBuf d_runs, d_shapes, d_first, d_wstart;
  int32_t add_shape(const tk::SkRunShape& sh) {
    const std::string key(reinterpret_cast<const char*>(&sh), sizeof(sh));
    auto it = shape_id.find(key);
    if (it != shape_id.end()) return it->second;
    if (shapes.size() >= static_cast<size_t>(INT32_MAX)) fail(TK_ERR_UNSUPPORTED, "too many run shapes");
    const int32_t id = static_cast<int32_t>(shapes.size());
    shapes.push_back(sh);
    shape_id.emplace(key, id);
    return id;
  }
  void finalize() {
    std::sort(runs.begin(), runs.end(), [](const tk::SkRun& x, const tk::SkRun& y) {
      return x.buf != y.buf ? x.buf < y.buf : x.off < y.off;
    });
    if (runs.size() > static_cast<size_t>(INT32_MAX) || shapes.size() > static_cast<size_t>(INT32_MAX))
      fail(TK_ERR_UNSUPPORTED, "too many output runs");
    total = 0;
    for (auto& r : runs) {
      r.vstart = total;
      total += r.len;
    }
    first.clear();
    wstart.clear();
    if (runs.empty()) return;
    int64_t v = 0;
    size_t r = 0;
    wstart.push_back(0);
    first.push_back(0);
    while (v < total) {
      int64_t stop = std::min(total, v + tk::kRunChunk);
      if (r + tk::kRunMax < runs.size()) stop = std::min(stop, runs[r + tk::kRunMax].vstart);
      v = stop;
      while (r + 1 < runs.size() && runs[r + 1].vstart <= v) ++r;
      wstart.push_back(v);
      first.push_back(static_cast<int32_t>(r));
    }
    if (wstart.size() - 1 > static_cast<size_t>(INT32_MAX)) fail(TK_ERR_UNSUPPORTED, "too many output-run workgroups");
    std::vector<int64_t> vs(runs.size());
    for (size_t i = 0; i < runs.size(); ++i) {
      const tk::SkRun& rn = runs[i];
      vs[i] = rn.vstart;
      if (rn.shape < 0 || rn.shape >= static_cast<int32_t>(shapes.size()))
        fail(TK_ERR_UNSUPPORTED, "output run with a bad dimension record");
      const tk::SkRunShape& sh = shapes[rn.shape];
      if (sh.nd < 0 || sh.nd > 8) fail(TK_ERR_UNSUPPORTED, "output-run record with more than 8 dimensions");
      int64_t cap = 1;
      for (int o = 0; o < sh.nd; ++o) cap *= sh.dim[o].dimshr & 0xffffff;
      if (rn.lin0 < 0 || rn.lin0 + static_cast<int64_t>(rn.len) > cap)
        fail(TK_ERR_UNSUPPORTED, "output run reaches past its block");
    }
    check_chunks(vs, total, first, wstart, tk::kRunChunk, tk::kRunMax, "output-run");
  }
  int nwg() const { return wstart.empty() ? 0 : static_cast<int>(wstart.size()) - 1; }
  void upload() {
    d_runs.upload(runs);
    d_shapes.upload(shapes);
    d_first.upload(first);
    d_wstart.upload(wstart);
  }
};

// Small-K tasks of one K value (one workgroup each).
struct SmallKSet {
  std::vector<tk::SmallKTask> tasks;
  DevBuf d_tasks;
  int n() const { return static_cast<int>(tasks.size()); }
  void upload() { d_tasks.upload(tasks); }
};

int32_t checked_i32(int64_t v, const char* what) {
  if (v > INT32_MAX || v < INT32_MIN) fail(TK_ERR_UNSUPPORTED, std::string(what) + " exceeds 32 bits");
  return static_cast<int32_t>(v);
}

// Multiply-high form of division by d (1 <= d < 2^31) for dividends below
// 2^31 (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): with l = ceil(log2 d) and M = floor(2^(31+l)/d) + 1,
// floor(x M / 2^(31+l)) = floor(x / d), since the error M - 2^(31+l)/d lies in
// (0, 1] and so adds less than x / 2^(31+l) < 1/d.  M < 2^32.
void division_magic(uint32_t d, uint32_t* mag, uint8_t* shr) {
  int l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  const int k = 31 + l;
  *mag = static_cast<uint32_t>((uint64_t(1) << k) / d + 1);
  *shr = static_cast<uint8_t>(k);
}

// Output runs of one small-K sector whose blocks land in C: one decoder per
// block (row channel i x column channel j) and one run per stretch of the
// block that is contiguous in C (the leading output dimensions whose strides
// are those of a dense array).  Returns false, adding nothing, when the runs
// would be short (under 4 elements on average) or a block does not fit the
// decoder's 24-bit arithmetic (2^24 elements or more, an operand offset or
// the A~ column stride 2^24 or more).
bool add_output_runs(RunSet& rs, const Structure& Ct, const Group& rg, const Group& cg,
                     const std::vector<tk::SkChan>& chans, int32_t rbase, int32_t cbase,
                     const std::vector<PairDesc>& pairs, int32_t pbase, const std::vector<int>& src, bool scatter,
                     int64_t a0, int64_t b0, int64_t M, int64_t K, int16_t abuf, int16_t bbuf) {
  const int nrow = scatter ? Ct.N1() : 1;
  const int nout = scatter ? Ct.N() : 2;
  struct Blk {
    int64_t dim[8], str[8], so[8];
    uint32_t bmask;
    int64_t runlen, count;
  };
  std::vector<Blk> blks(static_cast<size_t>(rg.n()) * cg.n());
  int64_t nruns = 0, nelem = 0;
  for (int32_t i = 0; i < rg.n(); ++i)
    for (int32_t j = 0; j < cg.n(); ++j) {
      const tk::SkChan& rc = chans[rbase + i];
      const tk::SkChan& cc = chans[cbase + j];
      const PairDesc& pd = pairs[pbase + i * cg.n() + j];
      Blk& b = blks[static_cast<size_t>(i) * cg.n() + j];
      b.bmask = 0;
      for (int n = 0; n < 8; ++n) {
        b.dim[n] = 1;
        b.str[n] = 0;
        b.so[n] = 0;
      }
      for (int n = 0; n < nout; ++n) {
        const int l = scatter ? src[n] : n;
        if (l < nrow) {
          int64_t st = 1;
          for (int q = 0; q < l; ++q) st *= rc.dim[q];
          b.dim[n] = rc.dim[l];
          b.str[n] = st;
          b.so[n] = pd.S[l];
        } else {
          const int m = l - nrow;
          int64_t st = K;
          for (int q = 0; q < m; ++q) st *= cc.dim[q];
          b.dim[n] = cc.dim[m];
          b.str[n] = st;
          b.so[n] = pd.S[4 + m];
          b.bmask |= 1u << n;
        }
      }
      b.count = int64_t(rc.count) * cc.count;
      int64_t amax = 0, bmax = 0;
      for (int n = 0; n < nout; ++n) ((b.bmask >> n) & 1u ? bmax : amax) += (b.dim[n] - 1) * b.str[n];
      if (b.count >= kRunLimit || amax >= kRunLimit || bmax >= kRunLimit) return false;
      int64_t run = 1;
      for (int n = 0; n < nout && (b.dim[n] == 1 || b.so[n] == run); ++n) run *= b.dim[n];
      b.runlen = run;
      nruns += b.count / run;
      nelem += b.count;
    }
  if (nruns * 4 > nelem || M >= kRunLimit) return false;
  for (int32_t i = 0; i < rg.n(); ++i)
    for (int32_t j = 0; j < cg.n(); ++j) {
      const size_t bi = static_cast<size_t>(i) * cg.n() + j;
      const Blk& b = blks[bi];
      const PairDesc& pd = pairs[pbase + i * cg.n() + j];
      tk::SkRunShape sh{};
      for (int n = 0; n < 8; ++n) {
        if (b.dim[n] == 1) continue;  // its index is always 0
        uint32_t mag = 0;
        uint8_t shr = 0;
        division_magic(static_cast<uint32_t>(b.dim[n]), &mag, &shr);  // shr >= 32 for extents >= 2
        tk::SkRunDim& o = sh.dim[sh.nd++];
        o.mag = mag;
        o.dimshr = static_cast<uint32_t>(b.dim[n]) | (static_cast<uint32_t>(shr - 32) << 24);
        o.sa = (b.bmask >> n) & 1u ? 0u : static_cast<uint32_t>(b.str[n]);
        o.sb = (b.bmask >> n) & 1u ? static_cast<uint32_t>(b.str[n]) : 0u;
      }
      const int32_t shape = rs.add_shape(sh);
      for (int64_t lin0 = 0; lin0 < b.count; lin0 += b.runlen) {
        tk::SkRun r{};
        int64_t rem = lin0, x = 0;
        for (int n = 0; n < 8; ++n) {
          x += (rem % b.dim[n]) * b.so[n];
          rem /= b.dim[n];
        }
        r.off = pd.base + x;
        r.a = a0 + rg.off[i];
        r.b = b0 + cg.off[j] * K;
        r.lin0 = static_cast<int32_t>(lin0);
        r.shape = shape;
        r.lda = checked_i32(M, "M");
        r.sign = pd.sign;
        r.buf = tk::kBufC;
        r.a_buf = abuf;
        r.b_buf = bbuf;
        r.len = static_cast<int32_t>(b.runlen);
        rs.runs.push_back(r);
      }
    }
  return true;
}

// Add one block (dims/strides in output order) as chunked tasks.
// Blocks whose source and destination are contiguous along different
// dimensions, both at least this long, are permuted through LDS tiles.
constexpr int64_t kTileMinEdge = 16;

void add_block_tasks(TaskList& tl, int16_t sbuf, int64_t src, int16_t dbuf, int64_t dst, int n, const int64_t* dim,
                     const int64_t* ss, const int64_t* ds, float sign, int32_t lo = 0) {
  // drop unit dims, merge dims that are contiguous on both sides
  int64_t D[tk::kMaxDims], S[tk::kMaxDims], T[tk::kMaxDims];
  int m = 0;
  for (int i = 0; i < n; ++i) {
    if (dim[i] == 1) continue;
    if (m > 0 && ss[i] == S[m - 1] * D[m - 1] && ds[i] == T[m - 1] * D[m - 1]) {
      D[m - 1] *= dim[i];
      continue;
    }
    D[m] = dim[i];
    S[m] = ss[i];
    T[m] = ds[i];
    ++m;
  }
  if (m == 0) {
    D[0] = 1;
    S[0] = 0;
    T[0] = 0;
    m = 1;
  }
  int64_t total = 1;
  for (int i = 0; i < m; ++i) total *= D[i];
  if (total > INT32_MAX) fail(TK_ERR_UNSUPPORTED, "block larger than 2^31 elements");
  // source contiguous along dim a, destination along dim b != a: tiles of
  // kTileEdge x kTileEdge through LDS at every index of the other dims
  int a = -1, b = -1;
  for (int i = 0; i < m; ++i) {
    if (S[i] == 1 && a < 0) a = i;
    if (T[i] == 1 && b < 0) b = i;
  }
  if (sbuf >= 0 && a >= 0 && b >= 0 && a != b && D[a] >= kTileMinEdge && D[b] >= kTileMinEdge) {
    int64_t idx[tk::kMaxDims] = {0};
    const int64_t E = tk::kTileEdge;
    for (;;) {
      int64_t so = src, dof = dst;
      for (int i = 0; i < m; ++i)
        if (i != a && i != b) {
          so += idx[i] * S[i];
          dof += idx[i] * T[i];
        }
      for (int64_t ia = 0; ia < D[a]; ia += E)
        for (int64_t ib = 0; ib < D[b]; ib += E) {
          tk::TileTask t{};
          t.src = so + ia + ib * S[b];
          t.dst = dof + ia * T[a] + ib;
          t.ea = static_cast<int32_t>(std::min(E, D[a] - ia));
          t.eb = static_cast<int32_t>(std::min(E, D[b] - ib));
          t.sb = checked_i32(S[b], "stride");
          t.ta = checked_i32(T[a], "stride");
          t.src_buf = sbuf;
          t.dst_buf = dbuf;
          t.sign = sign;
          t.lo = lo;
          tl.tiles.push_back(t);
        }
      int i = 0;
      for (; i < m; ++i) {
        if (i == a || i == b) continue;
        if (++idx[i] < D[i]) break;
        idx[i] = 0;
      }
      if (i == m) break;
    }
    if (tl.tiles.size() > static_cast<size_t>(INT32_MAX)) fail(TK_ERR_UNSUPPORTED, "too many permute tiles");
    return;
  }
  // The kernel forms element offsets in 32 bits, relative to the task's
  // source and destination.  A block whose offsets span 2^31 or more (a
  // small block inside a huge sector) is cut along its outermost dims into
  // slices that fit, each with its own 64-bit base.
  std::function<void(int64_t, int64_t, int)> emit = [&](int64_t so, int64_t dof, int md) {
    int64_t sspan = 0, dspan = 0, cnt = 1;
    for (int i = 0; i < md; ++i) {
      sspan += (D[i] - 1) * S[i];
      dspan += (D[i] - 1) * T[i];
      cnt *= D[i];
    }
    if (sspan > INT32_MAX || dspan > INT32_MAX) {
      for (int64_t x = 0; x < D[md - 1]; ++x) emit(so + x * S[md - 1], dof + x * T[md - 1], md - 1);
      return;
    }
    PermTask t{};
    t.lo = lo;
    t.src = so;
    t.dst = dof;
    t.n = std::max(md, 1);
    t.src_buf = sbuf;
    t.dst_buf = dbuf;
    t.sign = sign;
    for (int i = 0; i < tk::kMaxDims; ++i) {
      t.dim[i] = i < md ? checked_i32(D[i], "dim") : 1;
      t.ss[i] = i < md ? checked_i32(S[i], "stride") : 0;
      t.ds[i] = i < md ? checked_i32(T[i], "stride") : 0;
      division_magic(static_cast<uint32_t>(t.dim[i]), &t.mag[i], &t.shr[i]);
    }
    for (int64_t s0 = 0; s0 < cnt; s0 += tk::kPermChunk) {
      t.start = static_cast<int32_t>(s0);
      t.count = static_cast<int32_t>(std::min<int64_t>(tk::kPermChunk, cnt - s0));
      tl.tasks.push_back(t);
    }
  };
  emit(src, dst, m);
}

// Sector GEMMs with K at most this run as an output-stationary stream.
constexpr int64_t kSmallK = 8;
// columns per small-K task
constexpr int64_t kSkCols = 64;
// elements per strip of whole small-K output blocks
constexpr int64_t kSkStrip = 16384;

// Add one output block of a small-K sector GEMM (dims and strides in output
// leg order) as chunked tasks, merging dims contiguous in r, s and dst.
// Pack consecutive tasks into workgroups of about kPermChunk elements.
// Tasks of one workgroup at most: one per wave, so small tasks (a handful
// of elements each) run side by side instead of one after another.
constexpr int kTasksPerWg = 4;

template <typename TL>
void pack_workgroups(TL& tl, int64_t limit = tk::kPermChunk) {
  tl.wg_first.assign(1, 0);
  int64_t acc = 0;
  int ntask = 0;
  for (size_t i = 0; i < tl.tasks.size(); ++i) {
    const int c = tl.tasks[i].count;
    if (ntask > 0 && (acc + c > limit || ntask >= kTasksPerWg)) {
      tl.wg_first.push_back(static_cast<int32_t>(i));
      acc = 0;
      ntask = 0;
    }
    acc += c;
    ++ntask;
  }
  if (!tl.tasks.empty()) tl.wg_first.push_back(static_cast<int32_t>(tl.tasks.size()));
}

// Strides of a block inside its coupled-charge matrix, per leg.
void block_strides(const Structure& st, const uint8_t* tup, int64_t R, int64_t* dims, int64_t* strides) {
  int64_t acc = 1;
  for (int l = 0; l < st.N1(); ++l) {
    dims[l] = st.leg(l).deg[tup[l]];
    strides[l] = acc;
    acc *= dims[l];
  }
  acc = R;
  for (int l = st.N1(); l < st.N(); ++l) {
    dims[l] = st.leg(l).deg[tup[l]];
    strides[l] = acc;
    acc *= dims[l];
  }
}

struct BlockLoc {
  int sector = -1;
  int32_t row = -1, col = -1;
  int64_t offset = 0, R = 0;
};

// Locate the block of `st` with leg sector indices tup (codomain then domain).
BlockLoc locate(const Structure& st, const uint8_t* tup) {
  BlockLoc b;
  const int64_t key = st.tuple_key(st.cod, tup);
  b.sector = st.sector_of_key(key);
  if (b.sector < 0) return b;
  b.row = st.rows.find(tup);
  b.col = st.cols.find(tup + st.N1());
  if (b.row < 0 || b.col < 0) {
    b.sector = -1;
    return b;
  }
  b.R = st.R[b.sector];
  b.offset = st.soff[b.sector] + st.cg[b.sector]->off[b.col] * b.R + st.rg[b.sector]->off[b.row];
  return b;
}

// Iterate the blocks of a structure in storage order.
template <typename F>
void for_each_block(const Structure& st, F&& f) {
  std::vector<uint8_t> tup(st.N());
  for (size_t s = 0; s < st.keys.size(); ++s) {
    const Group& rg = *st.rg[s];
    const Group& cg = *st.cg[s];
    for (int32_t j = 0; j < cg.n(); ++j) {
      std::copy(cg.idx.begin() + size_t(j) * st.N2(), cg.idx.begin() + size_t(j + 1) * st.N2(), tup.begin() + st.N1());
      for (int32_t i = 0; i < rg.n(); ++i) {
        std::copy(rg.idx.begin() + size_t(i) * st.N1(), rg.idx.begin() + size_t(i + 1) * st.N1(), tup.begin());
        const int64_t off = st.soff[s] + cg.off[j] * st.R[s] + rg.off[i];
        f(static_cast<int>(s), i, j, tup.data(), off);
      }
    }
  }
}

int channel_parity(const Structure& st, const uint8_t* tup, const std::vector<std::pair<int, int>>& pairs) {
  int s = 0;
  for (const auto& pr : pairs) s ^= (st.leg(pr.first).p[tup[pr.first]] & st.leg(pr.second).p[tup[pr.second]]);
  return s;
}

// Permute plan A -> C (Alg. "Abelian Tensor Permutation"); twist additionally
// multiplies by (-1)^{|x|} for every codomain leg of C on a dual space.
// Split-BF16x3 operand planes of a permuted operand (the structure C of
// plan_permute_tasks): per sector of C its first element in the planes (-1:
// the sector is not split and keeps its place in the buffer dbuf, or is
// skipped when dbuf < 0), the padded length ld of a row (rows: A~, element
// (r, c) at off + r ld + c) or of a column (B~: off + r + c ld), the buffer of
// the hi plane and the lo plane's distance from it.
struct PlaneMap {
  std::vector<int64_t> off, ld;
  bool rows = false;
  int16_t buf = 0;
  int32_t lo = 0;
};

void plan_permute_tasks(const Structure& A, const std::vector<int>& p, const std::vector<int>& q, const Structure& C,
                        int16_t sbuf, int16_t dbuf, bool twist, TaskList& tl, std::vector<int64_t>* map_out = nullptr,
                        std::vector<int32_t>* sign_out = nullptr, const PlaneMap* planes = nullptr) {
  const bool ferm = A.si.fermionic;
  const auto pairs = ferm ? exchanged_pairs(A.N1(), A.N2(), p, q) : std::vector<std::pair<int, int>>{};
  std::vector<int> src(p);
  src.insert(src.end(), q.begin(), q.end());
  const int N = A.N();
  std::vector<uint8_t> otup(N);
  int64_t idim[TK_MAX_RANK], istr[TK_MAX_RANK], odim[TK_MAX_RANK], ostr[TK_MAX_RANK], oss[TK_MAX_RANK];
  for_each_block(A, [&](int s, int32_t, int32_t, const uint8_t* tup, int64_t off) {
    for (int n = 0; n < N; ++n) otup[n] = tup[src[n]];
    const BlockLoc b = locate(C, otup.data());
    if (b.sector < 0) fail(TK_ERR_SPACE_MISMATCH, "permute: output tensor lacks a channel of the input");
    block_strides(A, tup, A.R[s], idim, istr);
    block_strides(C, otup.data(), b.R, odim, ostr);
    for (int n = 0; n < N; ++n) oss[n] = istr[src[n]];
    int par = ferm ? channel_parity(A, tup, pairs) : 0;
    if (twist && ferm)
      for (int n = 0; n < C.N1(); ++n)
        if (C.cod[n].dual) par ^= C.cod[n].p[otup[n]];
    const float sign = par ? -1.0f : 1.0f;
    if (map_out) {
      map_out->push_back(C.bbase[b.sector] + static_cast<int64_t>(b.col) * C.rg[b.sector]->n() + b.row);
      sign_out->push_back(par ? -1 : 1);
      return;
    }
    if (planes && planes->off[b.sector] >= 0) {
      // the block in the planes: rows of A~ or columns of B~ of length ld
      const int64_t ld = planes->ld[b.sector];
      const int64_t r0 = C.rg[b.sector]->off[b.row], c0 = C.cg[b.sector]->off[b.col];
      int64_t pstr[TK_MAX_RANK];
      for (int n = 0; n < N; ++n) {
        const bool row_leg = n < C.N1();
        const int64_t unit = row_leg ? ostr[n] : ostr[n] / b.R;  // stride in rows / in columns
        pstr[n] = planes->rows ? (row_leg ? unit * ld : unit) : (row_leg ? unit : unit * ld);
      }
      const int64_t dst = planes->off[b.sector] + (planes->rows ? r0 * ld + c0 : r0 + c0 * ld);
      add_block_tasks(tl, sbuf, off, planes->buf, dst, N, odim, oss, pstr, sign, planes->lo);
      return;
    }
    if (dbuf < 0) return;
    add_block_tasks(tl, sbuf, off, dbuf, b.offset, N, odim, oss, ostr, sign);
  });
}

// Zero padding of split planes: in every split sector the k range K .. ld-1
// of each of its n rows (A~) or columns (B~).
void plan_plane_padding(const Structure& C, const PlaneMap& pm, TaskList& tl) {
  for (size_t s = 0; s < C.keys.size(); ++s) {
    if (pm.off[s] < 0) continue;
    const int64_t K = pm.rows ? C.C[s] : C.R[s], n = pm.rows ? C.R[s] : C.C[s], pad = pm.ld[s] - K;
    if (pad <= 0) continue;
    const int64_t dim[2] = {pad, n}, zs[2] = {0, 0}, ds[2] = {1, pm.ld[s]};
    add_block_tasks(tl, -1, 0, pm.buf, pm.off[s] + K, 2, dim, zs, ds, 1.0f, pm.lo);
  }
}

// Partial trace (Alg. "Abelian Tensor Trace"): legs t1[i] and t2[i] of A are
// closed with each other, the free legs form C's codomain p and domain q.
bool lin_dual(const Structure& A, int l) { return A.leg(l).dual != (l >= A.N1()); }

void check_trace_lists(const Structure& A, const std::vector<int>& p, const std::vector<int>& q,
                       const std::vector<int>& t1, const std::vector<int>& t2) {
  const int N = A.N();
  if (t1.empty() || t1.size() != t2.size()) fail(TK_ERR_INVALID_ARG, "a trace needs matching, non-empty leg pair lists");
  if (t1.size() > static_cast<size_t>(tk::kMaxTracePairs)) fail(TK_ERR_UNSUPPORTED, "more than 4 traced leg pairs");
  std::vector<char> seen(N, 0);
  for (const auto* v : {&p, &q, &t1, &t2})
    for (int x : *v) {
      if (x < 0 || x >= N || seen[x]) fail(TK_ERR_INVALID_ARG, "(p, q, t1, t2) must list every leg exactly once");
      seen[x] = 1;
    }
  if (static_cast<int>(p.size() + q.size() + t1.size() + t2.size()) != N)
    fail(TK_ERR_INVALID_ARG, "(p, q, t1, t2) must list every leg exactly once");
  if (p.size() > TK_MAX_LEGS || q.size() > TK_MAX_LEGS) fail(TK_ERR_UNSUPPORTED, "too many legs on one side");
  for (size_t i = 0; i < t1.size(); ++i) {
    const Space &x = A.leg(t1[i]), &y = A.leg(t2[i]);
    if (x.q != y.q || x.p != y.p || x.deg != y.deg) fail(TK_ERR_SPACE_MISMATCH, "traced legs carry different spaces");
    if (lin_dual(A, t1[i]) == lin_dual(A, t2[i]))
      fail(TK_ERR_SPACE_MISMATCH, "traced legs are not a vector / co-vector pair");
  }
}

// Leg pairs whose order flips between A's bra-ket reading (codomain, then
// domain reversed) and the order in which the graph closes the trace: each
// traced pair adjacent with its dual (in that reading) leg first, then the
// free legs in C's bra-ket reading.
std::vector<std::pair<int, int>> trace_exchanged_pairs(const Structure& A, const std::vector<int>& p,
                                                       const std::vector<int>& q, const std::vector<int>& t1,
                                                       const std::vector<int>& t2) {
  const int N1 = A.N1(), N = A.N();
  std::vector<int> pos_in(N), pos_out(N), target;
  for (int l = 0; l < N1; ++l) pos_in[l] = l;
  for (int l = N1; l < N; ++l) pos_in[l] = N - 1 - (l - N1);
  for (size_t i = 0; i < t1.size(); ++i) {
    const bool xd = lin_dual(A, t1[i]);
    target.push_back(xd ? t1[i] : t2[i]);
    target.push_back(xd ? t2[i] : t1[i]);
  }
  target.insert(target.end(), p.begin(), p.end());
  target.insert(target.end(), q.rbegin(), q.rend());
  for (int k = 0; k < N; ++k) pos_out[target[k]] = k;
  std::vector<std::pair<int, int>> r;
  for (int x = 0; x < N; ++x)
    for (int y = 0; y < N; ++y)
      if (pos_in[x] < pos_in[y] && pos_out[x] > pos_out[y]) r.emplace_back(x, y);
  return r;
}

// output elements per trace task: one pass of a 256-thread workgroup at 4
// elements per thread, and small, so that a trace with few large output
// blocks still spreads over every CU
constexpr int64_t kTraceChunk = 1024;

struct TracePlan {
  std::shared_ptr<Structure> A, C;
  TaskListT<tk::TraceTask> tl;
  std::vector<tk::TraceContrib> contribs;
  DevBuf d_contribs;
};

void plan_trace_tasks(const Structure& A, const std::vector<int>& p, const std::vector<int>& q,
                      const std::vector<int>& t1, const std::vector<int>& t2, const Structure& C, TracePlan& tp) {
  const bool ferm = A.si.fermionic;
  const auto pairs = ferm ? trace_exchanged_pairs(A, p, q, t1, t2) : std::vector<std::pair<int, int>>{};
  std::vector<int> src(p);
  src.insert(src.end(), q.begin(), q.end());
  const int n = static_cast<int>(src.size()), nt = static_cast<int>(t1.size());
  std::vector<uint8_t> otup(std::max(n, 1));
  int64_t idim[TK_MAX_RANK], istr[TK_MAX_RANK], odim[TK_MAX_RANK], ostr[TK_MAX_RANK];
  std::unordered_map<int64_t, std::vector<tk::TraceContrib>> by_block;  // output block offset -> inputs
  for_each_block(A, [&](int s, int32_t, int32_t, const uint8_t* tup, int64_t off) {
    for (int k = 0; k < nt; ++k)
      if (tup[t1[k]] != tup[t2[k]]) return;  // the pairing is diagonal in the sector
    for (int m = 0; m < n; ++m) otup[m] = tup[src[m]];
    const BlockLoc b = locate(C, otup.data());
    if (b.sector < 0) fail(TK_ERR_SPACE_MISMATCH, "internal: C lacks a channel of the trace");
    block_strides(A, tup, A.R[s], idim, istr);
    tk::TraceContrib c{};
    c.src = off;
    c.coef = (ferm && channel_parity(A, tup, pairs)) ? -1.0 : 1.0;
    c.nd = nt;
    for (int m = 0; m < n; ++m) c.ss[m] = checked_i32(istr[src[m]], "stride");
    for (int k = 0; k < nt; ++k) {
      c.dd[k] = checked_i32(idim[t1[k]], "degeneracy");
      c.dstr[k] = checked_i32(istr[t1[k]] + istr[t2[k]], "stride");
    }
    by_block[b.offset].push_back(c);
  });
  for_each_block(C, [&](int s, int32_t, int32_t, const uint8_t* ot, int64_t off) {
    block_strides(C, ot, C.R[s], odim, ostr);
    const int32_t c0 = checked_i32(static_cast<int64_t>(tp.contribs.size()), "trace contributions");
    auto it = by_block.find(off);
    if (it != by_block.end()) tp.contribs.insert(tp.contribs.end(), it->second.begin(), it->second.end());
    const int32_t c1 = checked_i32(static_cast<int64_t>(tp.contribs.size()), "trace contributions");
    int64_t total = 1;
    for (int m = 0; m < n; ++m) total *= odim[m];
    if (total > INT32_MAX) fail(TK_ERR_UNSUPPORTED, "trace output block larger than 2^31 elements");
    for (int64_t s0 = 0; s0 < total; s0 += kTraceChunk) {
      tk::TraceTask t{};
      t.dst = off;
      t.n = n;
      t.start = static_cast<int32_t>(s0);
      t.count = static_cast<int32_t>(std::min<int64_t>(kTraceChunk, total - s0));
      t.c0 = c0;
      t.c1 = c1;
      t.src_buf = tk::kBufA;
      t.dst_buf = tk::kBufC;
      for (int m = 0; m < tk::kMaxDims; ++m) {
        t.dim[m] = m < n ? checked_i32(odim[m], "dim") : 1;
        t.ds[m] = m < n ? checked_i32(ostr[m], "stride") : 0;
        division_magic(static_cast<uint32_t>(t.dim[m]), &t.mag[m], &t.shr[m]);
      }
      tp.tl.tasks.push_back(t);
    }
  });
  pack_workgroups(tp.tl, kTraceChunk);
}

// ---------------------------------------------------------------------------
// SU(2) recoupling (Section "Non-abelian symmetries": canonical fusion and
// splitting trees; Section "Fusion Tree Manipulations": F- and R-moves;
// Alg. "Non-abelian Tensor Transformation").  Spins are twice their value.
// A permutation of legs within one side acts on a canonical splitting tree
// as a product of adjacent swaps; each swap is a local move built from the
// 6j symbols (F) and the exchange phases (R), so no dense Clebsch-Gordan
// tensors are formed.
// ---------------------------------------------------------------------------
namespace su2 {

long double fact_half(int n2) {  // (n2 / 2)!
  static const std::vector<long double> table = [] {
    std::vector<long double> t(171);
    t[0] = 1.0L;
    for (size_t i = 1; i < t.size(); ++i) t[i] = t[i - 1] * static_cast<long double>(i);
    return t;
  }();
  const int n = n2 / 2;
  if (n2 < 0 || (n2 & 1) || n >= static_cast<int>(table.size())) fail(TK_ERR_UNSUPPORTED, "spin too large");
  return table[n];
}

bool triangle(int a, int b, int c) { return std::abs(a - b) <= c && c <= a + b && ((a + b + c) & 1) == 0; }

long double delta(int a, int b, int c) {
  return std::sqrt(fact_half(a + b - c) * fact_half(a - b + c) * fact_half(-a + b + c) / fact_half(a + b + c + 2));
}

// Wigner 6j symbol {j1 j2 j3; j4 j5 j6} by Racah's single-sum formula.
double sixj(int j1, int j2, int j3, int j4, int j5, int j6) {
  if (!triangle(j1, j2, j3) || !triangle(j1, j5, j6) || !triangle(j4, j2, j6) || !triangle(j4, j5, j3)) return 0.0;
  const int a1 = j1 + j2 + j3, a2 = j1 + j5 + j6, a3 = j4 + j2 + j6, a4 = j4 + j5 + j3;
  const int b1 = j1 + j2 + j4 + j5, b2 = j2 + j3 + j5 + j6, b3 = j3 + j1 + j6 + j4;
  const int tmin = std::max(std::max(a1, a2), std::max(a3, a4)), tmax = std::min(b1, std::min(b2, b3));
  long double sum = 0.0L;
  for (int t = tmin; t <= tmax; t += 2) {
    const long double term = fact_half(t + 2) / (fact_half(t - a1) * fact_half(t - a2) * fact_half(t - a3) *
                                                 fact_half(t - a4) * fact_half(b1 - t) * fact_half(b2 - t) *
                                                 fact_half(b3 - t));
    sum += ((t / 2) & 1) ? -term : term;
  }
  return static_cast<double>(delta(j1, j2, j3) * delta(j1, j5, j6) * delta(j4, j2, j6) * delta(j4, j5, j3) * sum);
}

// F-move of splitting trees: the coefficient of the tree (e (a b)h) g in the
// tree ((e a)f b) g, with Condon-Shortley Clebsch-Gordan vertices.
double fmove(int e, int a, int b, int g, int f, int h) {
  const int ph = (e + a + b + g) / 2;
  return ((ph & 1) ? -1.0 : 1.0) * std::sqrt(static_cast<double>((f + 1) * (h + 1))) * sixj(e, a, f, b, g, h);
}

// R-move: exchanging the two outgoing legs of the vertex c -> a x b.
double rmove(int a, int b, int c) { return (((a + b - c) / 2) & 1) ? -1.0 : 1.0; }

// Swap of adjacent legs k, k+1 (k >= 1) with e = e_{k-1}, a = leg k,
// b = leg k+1, g = e_{k+1}: the tree with intermediate f becomes a sum over
// trees with intermediate f2, coefficient sum_h F(e,a,b,g;f,h) R(a,b;h)
// F(e,b,a,g;f2,h).
double swap_coeff(int e, int a, int b, int g, int f, int f2) {
  double v = 0.0;
  for (int h = std::abs(a - b); h <= a + b; h += 2) {
    if (!triangle(e, h, g)) continue;
    v += fmove(e, a, b, g, f, h) * rmove(a, b, h) * fmove(e, b, a, g, f2, h);
  }
  return v;
}

struct Leg {
  std::vector<int> tj;
  std::vector<int64_t> deg;
  bool dual = false;  // the leg carries the dual space (Z on its outer line)
};

struct Tree {
  std::vector<int> sec;  // sector index per leg
  std::vector<int> e;    // e_1 .. e_N (e_1 = first spin, e_N = coupled)
  int64_t r0 = 0, n = 1;
};

// One side: trees grouped by coupled spin, in storage order.
struct Side {
  std::map<int, std::vector<Tree>> by_c;
  std::map<std::pair<std::vector<int>, std::vector<int>>, std::pair<int, int>> index;  // (sec, e) -> (c, position)
};

void enumerate_trees(const std::vector<Leg>& legs, Side& side) {
  const int N = static_cast<int>(legs.size());
  std::vector<int> sec(N, 0);
  for (;;) {
    std::vector<int> outer(N);
    int64_t n = 1;
    for (int k = 0; k < N; ++k) {
      outer[k] = legs[k].tj[sec[k]];
      n *= legs[k].deg[sec[k]];
    }
    std::vector<std::vector<int>> found;
    std::vector<int> e{outer[0]};
    std::function<void(int)> rec = [&](int k) {
      if (k == N) {
        found.push_back(e);
        return;
      }
      const int prev = e.back();
      for (int f = std::abs(prev - outer[k]); f <= prev + outer[k]; f += 2) {
        e.push_back(f);
        rec(k + 1);
        e.pop_back();
      }
    };
    rec(1);
    // intermediates e_2..e_{N-1} colex: compare from the last one
    std::sort(found.begin(), found.end(), [&](const std::vector<int>& x, const std::vector<int>& y) {
      for (int k = N - 2; k >= 1; --k)
        if (x[k] != y[k]) return x[k] < y[k];
      return false;
    });
    for (auto& ee : found) {
      auto& lst = side.by_c[ee.back()];
      Tree t;
      t.sec = sec;
      t.e = ee;
      t.n = n;
      t.r0 = lst.empty() ? 0 : lst.back().r0 + lst.back().n;
      side.index[{sec, ee}] = {ee.back(), static_cast<int>(lst.size())};
      lst.push_back(std::move(t));
    }
    int k = 0;  // next outer tuple, colex (first leg fastest)
    for (; k < N; ++k) {
      if (++sec[k] < static_cast<int>(legs[k].tj.size())) break;
      sec[k] = 0;
    }
    if (k == N) break;
  }
}

struct Map {
  std::vector<Leg> cod, dom;
  Side rows, cols;
  std::map<int, std::array<int64_t, 3>> blocks;  // c -> offset, R, C
  int64_t size = 0;
  void build() {
    enumerate_trees(cod, rows);
    enumerate_trees(dom, cols);
    for (auto& [c, rl] : rows.by_c) {
      auto it = cols.by_c.find(c);
      if (it == cols.by_c.end()) continue;
      const int64_t R = rl.back().r0 + rl.back().n, C = it->second.back().r0 + it->second.back().n;
      blocks[c] = {size, R, C};
      size += R * C;
    }
  }
};

// The permuted tree (new leg k = old leg perm[k]) in canonical trees of the
// new outer spins: (new e sequence) -> coefficient.
std::map<std::vector<int>, double> permute_tree(const std::vector<int>& outer0, const std::vector<int>& e0,
                                                const std::vector<int>& perm) {
  const int N = static_cast<int>(outer0.size());
  std::vector<int> pos(N), cur(N);  // cur[k] = old leg now at position k
  for (int k = 0; k < N; ++k) {
    pos[perm[k]] = k;
    cur[k] = k;
  }
  std::map<std::vector<int>, double> v{{e0, 1.0}};
  bool moved = true;
  while (moved) {  // bubble sort by target position, one adjacent swap at a time
    moved = false;
    for (int k = 0; k + 1 < N; ++k) {
      if (pos[cur[k]] < pos[cur[k + 1]]) continue;
      const int a = outer0[cur[k]], b = outer0[cur[k + 1]];
      std::map<std::vector<int>, double> w;
      for (const auto& [e, x] : v) {
        if (k == 0) {
          std::vector<int> e2 = e;
          e2[0] = b;
          w[e2] += x * rmove(a, b, e[1]);
        } else {
          const int el = e[k - 1], g = e[k + 1];
          for (int f2 = std::abs(el - b); f2 <= el + b; f2 += 2) {
            if (!triangle(f2, a, g)) continue;
            const double cf = swap_coeff(el, a, b, g, e[k], f2);
            if (cf == 0.0) continue;
            std::vector<int> e2 = e;
            e2[k] = f2;
            w[e2] += x * cf;
          }
        }
      }
      v.swap(w);
      std::swap(cur[k], cur[k + 1]);
      moved = true;
    }
  }
  for (auto it = v.begin(); it != v.end();) it = std::fabs(it->second) < 1e-14 ? v.erase(it) : std::next(it);
  return v;
}


// Alg. "Non-abelian Tensor Transformation" as a gather: every output tree
// pair (s', f') collects, from each input pair (s, f) whose transform
// reaches it, the coefficient c_s c_f and the strides of the permuted input
// array; one trace-kernel task (no traced pairs) per chunk of an output pair
// sums them and writes each element once.
struct Plan {
  Map A, C;
  TaskListT<tk::TraceTask> tl;
  std::vector<tk::TraceContrib> contribs;
  std::vector<int64_t> tab_dst, tab_src;
  DevBuf d_contribs;
  int device = -1;
  bool gather = true;  // every output array's inputs share their strides
};

// Contributions by output tree pair (coupled spin, row tree, column tree):
// the input array (first element) with its strides in output leg order and
// the coefficient.
using Contribs = std::map<std::tuple<int, int, int>, std::vector<std::pair<tk::TraceContrib, int64_t>>>;

// Clebsch-Gordan coefficient <j1 m1, j2 m2 | J M> with Condon-Shortley
// phases (all arguments twice their value), by Racah's closed formula.
double cgc(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M || !triangle(j1, j2, J) || std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
  if (((j1 + m1) & 1) || ((j2 + m2) & 1) || ((J + M) & 1)) return 0.0;
  const long double pre = (J + 1) * fact_half(J + j1 - j2) * fact_half(J - j1 + j2) * fact_half(j1 + j2 - J) /
                          fact_half(j1 + j2 + J + 2) * fact_half(J + M) * fact_half(J - M) * fact_half(j1 - m1) *
                          fact_half(j1 + m1) * fact_half(j2 - m2) * fact_half(j2 + m2);
  long double sum = 0.0L;
  for (int k = 0; k <= j1 + j2; k += 2) {
    const int a[5] = {j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k};
    if (*std::min_element(a, a + 5) < 0) continue;
    long double den = fact_half(k);
    for (int x : a) den *= fact_half(x);
    sum += ((k / 2) & 1) ? -1.0L / den : 1.0L / den;
  }
  return static_cast<double>(std::sqrt(pre) * sum);
}

// Dense canonical splitting tree of outer spins o_1..o_N with e_1 = o_1,
// .., e_N = c: X[m_1, .., m_N, m_c] flat, first index fastest, index i of a
// spin j standing for m = j - i.
std::vector<double> tree_dense(const std::vector<int>& outer, const std::vector<int>& e) {
  const int N = static_cast<int>(outer.size());
  std::vector<double> T(static_cast<size_t>((outer[0] + 1) * (outer[0] + 1)), 0.0);
  for (int i = 0; i <= outer[0]; ++i) T[i + (outer[0] + 1) * i] = 1.0;  // [m_1, e_1]
  int64_t lead = outer[0] + 1;                                          // product of the outer dims so far
  for (int k = 1; k < N; ++k) {
    const int a = e[k - 1], b = outer[k], c = e[k];
    std::vector<double> U(static_cast<size_t>(lead * (b + 1) * (c + 1)), 0.0);
    for (int ie = 0; ie <= a; ++ie)
      for (int ib = 0; ib <= b; ++ib)
        for (int ic = 0; ic <= c; ++ic) {
          const double w = cgc(a, a - 2 * ie, b, b - 2 * ib, c, c - 2 * ic);
          if (w == 0.0) continue;
          const double* src = T.data() + static_cast<int64_t>(ie) * lead;
          double* dst = U.data() + (static_cast<int64_t>(ic) * (b + 1) + ib) * lead;
          for (int64_t x = 0; x < lead; ++x) dst[x] += w * src[x];
        }
    T.swap(U);
    lead *= b + 1;
  }
  return T;
}

// Dense tree pair X_s X_f^T summed over m_c: flat over the codomain then the
// domain legs (first fastest), with the isomorphism Z on dual legs: along
// such a leg entry i is (-1)^i times entry d - 1 - i (m goes to -m).
std::vector<double> pair_dense(const std::vector<int>& co, const std::vector<int>& es, const std::vector<int>& dout,
                               const std::vector<int>& ef, const std::vector<char>& dual) {
  const std::vector<double> X = tree_dense(co, es), Y = tree_dense(dout, ef);
  const int c = es.back();
  int64_t nr = 1, nc = 1;
  for (int x : co) nr *= x + 1;
  for (int x : dout) nc *= x + 1;
  std::vector<double> G(static_cast<size_t>(nr * nc), 0.0);
  for (int mc = 0; mc <= c; ++mc)
    for (int64_t j = 0; j < nc; ++j) {
      const double y = Y[j + nc * mc];
      if (y == 0.0) continue;
      for (int64_t i = 0; i < nr; ++i) G[i + nr * j] += X[i + nr * mc] * y;
    }
  std::vector<int> dims(co);
  dims.insert(dims.end(), dout.begin(), dout.end());
  int64_t stride = 1;
  for (size_t l = 0; l < dims.size(); ++l) {
    const int64_t d = dims[l] + 1;
    if (dual[l]) {
      std::vector<double> H(G.size());
      for (int64_t x = 0; x < static_cast<int64_t>(G.size()); ++x) {
        const int64_t i = (x / stride) % d, inew = d - 1 - i;
        H[x + (inew - i) * stride] = (inew & 1) ? -G[x] : G[x];
      }
      G.swap(H);
    }
    stride *= d;
  }
  return G;
}

// Elements per recoupling task: one pass of the gather kernel's 256-thread
// workgroup at 8 elements per thread (1024 and 4096 measured slower on the
// spin-1 two-site swap).
constexpr int64_t kSu2Chunk = 2048;

// Strides of the reduced array of tree t (legs of one side, first fastest),
// starting at base.
void tree_strides(const std::vector<Leg>& legs, const Tree& t, int64_t base, int64_t* out) {
  int64_t st = base;
  for (size_t k = 0; k < legs.size(); ++k) {
    out[k] = st;
    st *= legs[k].deg[t.sec[k]];
  }
}

// Contributions of a braid within each side: the coefficient of a pair is
// the product of its two trees' coefficients.
Contribs braid_contribs(const Plan& P, const std::vector<int>& p, const std::vector<int>& q) {
  const Map& A = P.A;
  const Map& C = P.C;
  const int N1 = static_cast<int>(A.cod.size()), N2 = static_cast<int>(A.dom.size()), n = N1 + N2;
  std::vector<int> qd(N2);
  for (int k = 0; k < N2; ++k) qd[k] = q[k] - N1;
  // per side: coupled spin -> per input tree the (output position, coefficient) list
  auto side_map = [](const std::vector<Leg>& legs, const Side& in, const Side& out, const std::vector<int>& perm) {
    std::map<int, std::vector<std::vector<std::pair<int, double>>>> res;
    const int N = static_cast<int>(legs.size());
    for (const auto& [c, trees] : in.by_c) {
      auto& lst = res[c];
      for (const Tree& t : trees) {
        std::vector<int> outer(N), nsec(N);
        for (int k = 0; k < N; ++k) outer[k] = legs[k].tj[t.sec[k]];
        for (int k = 0; k < N; ++k) nsec[k] = t.sec[perm[k]];
        std::vector<std::pair<int, double>> row;
        for (const auto& [e2, cf] : permute_tree(outer, t.e, perm)) {
          auto it = out.index.find({nsec, e2});
          if (it == out.index.end() || it->second.first != c) fail(TK_ERR_INVALID_ARG, "internal: SU(2) tree lost");
          row.emplace_back(it->second.second, cf);
        }
        lst.push_back(std::move(row));
      }
    }
    return res;
  };
  const auto rmap = side_map(A.cod, A.rows, C.rows, p);
  const auto cmap = side_map(A.dom, A.cols, C.cols, qd);
  Contribs by_out;
  for (const auto& [c, blk] : A.blocks) {
    const int64_t off = blk[0], R = blk[1];
    const auto& rows = A.rows.by_c.at(c);
    const auto& cols = A.cols.by_c.at(c);
    for (size_t i = 0; i < rows.size(); ++i)
      for (size_t j = 0; j < cols.size(); ++j) {
        int64_t is[TK_MAX_RANK], js[TK_MAX_RANK];
        tree_strides(A.cod, rows[i], 1, is);
        tree_strides(A.dom, cols[j], R, js);
        tk::TraceContrib cb{};
        cb.src = off + rows[i].r0 + cols[j].r0 * R;
        cb.nd = 0;
        for (int m = 0; m < n; ++m) cb.ss[m] = checked_i32(m < N1 ? is[p[m]] : js[qd[m - N1]], "stride");
        for (const auto& [si, cs] : rmap.at(c)[i])
          for (const auto& [fj, cf] : cmap.at(c)[j]) {
            cb.coef = cs * cf;
            by_out[{c, si, fj}].emplace_back(cb, cb.src);
          }
      }
  }
  return by_out;
}

// Tasks of the gather: one per chunk of every output tree pair, with the
// contributions that reach it (output pairs with the same outer sectors
// interleaved, see below).
void build_tasks(Plan& P, const Contribs& by_out) {
  const Map& C = P.C;
  const int N1 = static_cast<int>(C.cod.size()), N2 = static_cast<int>(C.dom.size()), n = N1 + N2;
  // Output pairs with the same outer sectors (they differ only in
  // intermediate spins) read the same input arrays at the same relative
  // offsets; their tasks are interleaved in runs of 8 chunks so that chunk k
  // of every such sibling lands on the same XCD (workgroups are dealt to the
  // 8 XCDs round-robin) at about the same time, and the shared inputs are
  // served from that XCD's L2.
  std::map<std::tuple<int, std::vector<int>, std::vector<int>>, size_t> group_of;
  std::vector<std::vector<std::vector<tk::TraceTask>>> groups;
  for (const auto& [c, blk] : C.blocks) {
    const int64_t off = blk[0], R = blk[1];
    const auto& rows = C.rows.by_c.at(c);
    const auto& cols = C.cols.by_c.at(c);
    for (size_t i = 0; i < rows.size(); ++i)
      for (size_t j = 0; j < cols.size(); ++j) {
        auto key = std::make_tuple(c, rows[i].sec, cols[j].sec);
        auto g = group_of.find(key);
        if (g == group_of.end()) {
          g = group_of.emplace(key, groups.size()).first;
          groups.emplace_back();
        }
        groups[g->second].emplace_back();
        auto& mine = groups[g->second].back();
        int64_t os[TK_MAX_RANK], od[TK_MAX_RANK];
        tree_strides(C.cod, rows[i], 1, os);
        tree_strides(C.dom, cols[j], R, os + N1);
        for (int m = 0; m < N1; ++m) od[m] = C.cod[m].deg[rows[i].sec[m]];
        for (int m = 0; m < N2; ++m) od[N1 + m] = C.dom[m].deg[cols[j].sec[m]];
        const int64_t dst = off + rows[i].r0 + cols[j].r0 * R;
        const int32_t c0 = checked_i32(static_cast<int64_t>(P.contribs.size()), "contributions");
        auto it = by_out.find({c, static_cast<int>(i), static_cast<int>(j)});
        if (it != by_out.end())
          for (const auto& [cb, src] : it->second) {
            // the gather kernel forms one source offset per element, which
            // needs every input of this output array to have the same
            // strides (true for braids: same outer sectors, same coupled
            // spin); a transpose can mix inputs of different coupled spins,
            // whose domain strides differ: then the plan uses the trace
            // kernel's per-contribution strides
            if (std::memcmp(cb.ss, it->second.front().first.ss, sizeof(cb.ss)) != 0) P.gather = false;
            P.contribs.push_back(cb);
            P.tab_dst.push_back(dst);
            P.tab_src.push_back(src);
          }
        const int32_t c1 = checked_i32(static_cast<int64_t>(P.contribs.size()), "contributions");
        const int64_t total = rows[i].n * cols[j].n;
        if (total > INT32_MAX) fail(TK_ERR_UNSUPPORTED, "SU(2) reduced array larger than 2^31 elements");
        for (int64_t s0 = 0; s0 < total; s0 += kSu2Chunk) {
          tk::TraceTask t{};
          t.dst = dst;
          t.n = n;
          t.start = static_cast<int32_t>(s0);
          t.count = static_cast<int32_t>(std::min<int64_t>(kSu2Chunk, total - s0));
          t.c0 = c0;
          t.c1 = c1;
          t.src_buf = tk::kBufA;
          t.dst_buf = tk::kBufC;
          for (int m = 0; m < tk::kMaxDims; ++m) {
            t.dim[m] = m < n ? checked_i32(od[m], "dim") : 1;
            t.ds[m] = m < n ? checked_i32(os[m], "stride") : 0;
            division_magic(static_cast<uint32_t>(t.dim[m]), &t.mag[m], &t.shr[m]);
          }
          mine.push_back(t);
        }
      }
  }
  constexpr size_t kRun = 8;  // one chunk per XCD
  for (const auto& sib : groups) {
    size_t nchunk = 0;
    for (const auto& tl : sib) nchunk = std::max(nchunk, tl.size());
    for (size_t b = 0; b < nchunk; b += kRun)
      for (const auto& tl : sib)
        for (size_t k = b; k < std::min(b + kRun, tl.size()); ++k) P.tl.tasks.push_back(tl[k]);
  }
  pack_workgroups(P.tl, kSu2Chunk);
}

void plan_permute(Plan& P, const std::vector<int>& p, const std::vector<int>& q) {
  build_tasks(P, braid_contribs(P, p, q));
}

// Contributions of a transpose (legs may cross between codomain and
// domain; order = output codomain legs then output domain legs, as input leg
// numbers): the coefficient of input pair (s, f) in output pair (s', f') is
// the overlap of the dense form of (s', f') with the dense form of (s, f)
// whose legs are reordered, divided by d_c' (tree pairs are orthonormal with
// norm d_c), i.e. the Clebsch-Gordan sum that the bending moves (with the Z
// isomorphisms on dual legs) and the recoupling moves evaluate.
Contribs transpose_contribs(const Plan& P, const std::vector<int>& order) {
  const Map& A = P.A;
  const Map& C = P.C;
  const int N1 = static_cast<int>(A.cod.size()), N = N1 + static_cast<int>(A.dom.size());
  const int M1 = static_cast<int>(C.cod.size());
  std::vector<const Leg*> in(N), outl(N);
  for (int k = 0; k < N; ++k) in[k] = k < N1 ? &A.cod[k] : &A.dom[k - N1];
  for (int k = 0; k < N; ++k) outl[k] = k < M1 ? &C.cod[k] : &C.dom[k - M1];
  std::vector<char> din(N), dout(N);
  for (int k = 0; k < N; ++k) {
    din[k] = in[k]->dual;
    dout[k] = outl[k]->dual;
  }
  std::map<std::vector<int>, std::vector<double>> out_dense;  // (outer sectors, e's) -> dense output pair
  Contribs by_out;
  for (const auto& [c, blk] : A.blocks) {
    const int64_t off = blk[0], R = blk[1];
    const auto& rows = A.rows.by_c.at(c);
    const auto& cols = A.cols.by_c.at(c);
    for (size_t i = 0; i < rows.size(); ++i)
      for (size_t j = 0; j < cols.size(); ++j) {
        std::vector<int> sec(N), spin(N);
        for (int k = 0; k < N; ++k) {
          sec[k] = k < N1 ? rows[i].sec[k] : cols[j].sec[k - N1];
          spin[k] = in[k]->tj[sec[k]];
        }
        std::vector<int> co(spin.begin(), spin.begin() + N1), dv(spin.begin() + N1, spin.end());
        const std::vector<double> G = pair_dense(co, rows[i].e, dv, cols[j].e, din);
        // the input pair with its legs in output order
        std::vector<int64_t> dim(N), istr(N);
        int64_t tot = 1;
        for (int k = 0; k < N; ++k) {
          dim[k] = spin[k] + 1;
          istr[k] = tot;
          tot *= dim[k];
        }
        std::vector<double> Gp(G.size());
        {
          std::vector<int64_t> ostr(N);
          int64_t st = 1;
          for (int m = 0; m < N; ++m) {
            ostr[order[m]] = st;
            st *= dim[order[m]];
          }
          std::vector<int64_t> idx(N, 0);
          for (int64_t x = 0; x < tot; ++x) {
            int64_t y = 0;
            for (int k = 0; k < N; ++k) y += idx[k] * ostr[k];
            Gp[y] = G[x];
            for (int k = 0; k < N; ++k) {
              if (++idx[k] < dim[k]) break;
              idx[k] = 0;
            }
          }
        }
        // output outer sectors and spins
        std::vector<int> osec(N), ospin(N);
        for (int m = 0; m < N; ++m) {
          osec[m] = sec[order[m]];
          ospin[m] = spin[order[m]];
        }
        std::vector<int> osc(osec.begin(), osec.begin() + M1), osd(osec.begin() + M1, osec.end());
        std::vector<int> oco(ospin.begin(), ospin.begin() + M1), odv(ospin.begin() + M1, ospin.end());
        // input strides in output leg order
        int64_t is[TK_MAX_RANK], js[TK_MAX_RANK];
        tree_strides(A.cod, rows[i], 1, is);
        tree_strides(A.dom, cols[j], R, js);
        tk::TraceContrib cb{};
        cb.src = off + rows[i].r0 + cols[j].r0 * R;
        cb.nd = 0;
        for (int m = 0; m < N; ++m) cb.ss[m] = checked_i32(order[m] < N1 ? is[order[m]] : js[order[m] - N1], "stride");
        for (const auto& [c2, orow] : C.rows.by_c) {
          auto cit = C.cols.by_c.find(c2);
          if (cit == C.cols.by_c.end() || !C.blocks.count(c2)) continue;
          for (size_t si = 0; si < orow.size(); ++si) {
            if (orow[si].sec != osc) continue;
            for (size_t fj = 0; fj < cit->second.size(); ++fj) {
              const Tree& ft = cit->second[fj];
              if (ft.sec != osd) continue;
              std::vector<int> key(osec);
              key.insert(key.end(), orow[si].e.begin(), orow[si].e.end());
              key.insert(key.end(), ft.e.begin(), ft.e.end());
              auto hit = out_dense.find(key);
              if (hit == out_dense.end()) hit = out_dense.emplace(key, pair_dense(oco, orow[si].e, odv, ft.e, dout)).first;
              const std::vector<double>& H = hit->second;
              double v = 0.0;
              for (size_t x = 0; x < H.size(); ++x) v += H[x] * Gp[x];
              v /= (c2 + 1);
              if (std::fabs(v) < 1e-13) continue;
              cb.coef = v;
              by_out[{c2, static_cast<int>(si), static_cast<int>(fj)}].emplace_back(cb, cb.src);
            }
          }
        }
      }
  }
  return by_out;
}

void plan_transpose(Plan& P, const std::vector<int>& order) { build_tasks(P, transpose_contribs(P, order)); }

}  // namespace su2

// Whether a block with these dims and strides fills one contiguous range
// (its non-unit dims, ordered by stride, are densely packed from stride 1);
// *span = number of elements.
bool contiguous_block(int n, const int64_t* dim, const int64_t* stride, int64_t* span) {
  std::vector<std::pair<int64_t, int64_t>> ds;  // (stride, dim)
  int64_t total = 1;
  for (int i = 0; i < n; ++i) {
    total *= dim[i];
    if (dim[i] > 1) ds.push_back({stride[i], dim[i]});
  }
  std::sort(ds.begin(), ds.end());
  int64_t expect = 1;
  for (const auto& x : ds) {
    if (x.first != expect) return false;
    expect *= x.second;
  }
  *span = total;
  return true;
}


}  // namespace

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct tk_context {
  int device = 0;
  int num_cu = 256;
  std::mutex mu;
  std::unordered_map<std::string, std::shared_ptr<tk_plan>> plans;
  std::unordered_map<std::string, std::shared_ptr<struct PermPlan>> perm_plans;
  std::unordered_map<std::string, std::shared_ptr<struct TracePlan>> trace_plans;
};

struct tk_tensor {
  tk_context* ctx = nullptr;
  std::shared_ptr<Structure> st;
  int dtype = TK_F64;
  void* data = nullptr;
  uint64_t bytes = 0;
  bool owns = false;
  ~tk_tensor() {
    if (owns && data) (void)hipFree(data);
  }
  size_t esize() const { return dtype == TK_F64 ? 8 : 4; }
};

struct PermPlan {
  std::shared_ptr<Structure> A, C;
  TaskList tl;
};

struct tk_plan {
  tk_context* ctx = nullptr;
  std::shared_ptr<Structure> A, B, C, At, Bt, Ct;
  std::vector<int> pA, qA, pB, qB, pAB, qAB;
  int precision = 0, dtype = 0;
  bool permA = false, permB = false, scatter = false, post = false;
  TaskList pre, zero, postp;
  // operand permutes of A and of B alone; filled only when both have work
  // (pre_owner: bit 0 A has permute work, bit 1 B has)
  TaskList preA, preB;
  int pre_owner = 0;
  std::vector<GemmDesc> descs;
  std::vector<LegMap> row_map, col_map;
  std::vector<PairDesc> pairs;
  DevBuf d_descs, d_rowmap, d_colmap, d_pairs;
  // tile schedule
  int tile_m = 128, tile_n = 128, tile_k = 16;
  std::vector<GemmTile> tiles;
  std::vector<int32_t> wg_first;
  DevBuf d_tiles, d_wg;
  int32_t ngroups = 0, nslots = 0;
  double makespan = 0;
  DevBuf d_partials, d_groups;
  std::vector<GemmTile> groups;
  ZeroSet zranges;       // zero-fill of empty-K blocks that are contiguous ranges
  SmallKSet smallk[9];  // indexed by K: row-stationary small-K tasks
  SkBlockList skblocks[9];  // indexed by K: output-stationary small-K tasks
  RunSet skruns[9];         // indexed by K: output runs of small-K sectors
  std::vector<tk::SkChan> skchans;  // row / column channels of the small-K sectors
  std::vector<PairDesc> skpairs;    // output placement of their channel pairs
  DevBuf d_skchans, d_skpairs;
  std::vector<int64_t> mnk;  // (M, N, K) of every sector GEMM with K > 0, MFMA or streamed
  DevBuf wsA, wsB, wsC;
  bool needA = false, needB = false;  // the A~ / B~ workspaces are written (some sector uses them)
  int64_t planeA = 0, planeB = 0;     // elements of one split-BF16x3 plane of A~ / B~
  DevBuf wsAp, wsBp;                  // hi then lo plane of A~ / B~
  double flops = 0;
  int64_t nzero = 0;
};

struct tk_batch {
  tk_context* ctx = nullptr;
  int n = 0, dtype = 0, precision = 0;
  double alpha = 1.0, beta = 0.0;
  TaskList pre, zero, postp;
  ZeroSet zranges;
  SmallKSet smallk[9];
  SkBlockList skblocks[9];
  RunSet skruns[9];
  std::vector<tk::SkChan> skchans;
  std::vector<PairDesc> skpairs;
  DevBuf d_skchans, d_skpairs;
  int32_t ngroups = 0, nslots = 0;
  DevBuf d_partials, d_groups;
  std::vector<GemmTile> groups;
  std::vector<GemmDesc> descs;
  std::vector<LegMap> row_map, col_map;
  std::vector<PairDesc> pairs;
  DevBuf d_descs, d_rowmap, d_colmap, d_pairs, d_tiles, d_wg, d_table;
  std::vector<std::unique_ptr<DevBuf>> ws;
  int tile_m = 128, tile_n = 128, tile_k = 16;
  std::vector<GemmTile> tiles;
  std::vector<int32_t> wg_first;
  double flops = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~tk_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

// LPT schedule of the tiles of a set of GEMMs over at most max_wg
// workgroups: work units sorted by cost (K stages) and each given to the
// least loaded group.  When the whole-K tiles balance badly (few tiles, long
// K), tiles are split along K; the schedule with the smaller estimated
// makespan (including the partial-tile write and reduction of split units)
// is kept.
struct Sched {
  std::vector<GemmTile> tiles;
  std::vector<int32_t> wg_first;
  std::vector<GemmTile> groups;  // one descriptor per split group (its split 0)
  int32_t ngroups = 0, nslots = 0;
  double makespan = 0;
};

// Relative MFMA time of a tile whose valid extent is (mrem, nrem) rows and
// columns: waves of the GEMM kernel whose sub-tile is empty skip their MFMAs,
// and the tile takes as long as its busiest SIMD (waves w and w + NW/2 share
// one; the placement mirrors wave_origin in the kernel).
double tile_activity(int tm, int tn, int64_t mrem, int64_t nrem) {
  const int wgm = 2, wgn = (tm == 128 && tn == 128) || (tm == 64 && tn == 128) ? 4 : 2;
  const int nw = wgm * wgn, wmsz = tm / wgm, wnsz = tn / wgn;
  auto origin = [&](int w, int* wm, int* wn) {
    const int half = nw / 2, r = w / half, c = w % half;
    *wm = r * wmsz;
    *wn = ((c + r * (half / 2)) % half) * wnsz;
  };
  int busiest = 0;
  for (int simd = 0; simd < 4; ++simd) {
    int act = 0;
    for (int w = simd; w < nw; w += 4) {
      int wm, wn;
      origin(w, &wm, &wn);
      act += (wm < mrem && wn < nrem) ? 1 : 0;
    }
    busiest = std::max(busiest, act);
  }
  const int per_simd = (nw + 3) / 4;
  return double(busiest) / per_simd;
}

// XCDs of the device: workgroups are dispatched round robin over them.
constexpr int kNumXcd = 8;

// Work units of the tiles, each tagged with a cluster: a block of bm x bn
// tiles of one sector GEMM, which shares bm row panels of A and bn column
// panels of B.  Tiles are generated cluster by cluster, so that the units
// dealt out together to the CUs of one XCD (and run at the same time) read
// the same panels through that XCD's L2.
struct Unit {
  GemmTile t;
  int64_t cost;
};

std::vector<Unit> make_units(const std::vector<GemmDesc>& descs, int tm, int tn, int BK, int64_t split_target,
                             int bm, int bn, Sched& out) {
  std::vector<Unit> units;
  for (size_t g = 0; g < descs.size(); ++g) {
    const GemmDesc& d = descs[g];
    const int64_t stages = (d.K + BK - 1) / BK;
    int64_t S = 1;
    if (split_target > 0 && stages > split_target) {
      S = std::min<int64_t>((stages + split_target - 1) / split_target, 16);
      S = std::min<int64_t>(S, std::max<int64_t>(1, stages / 4));
    }
    const int mt = (d.M + tm - 1) / tm, nt = (d.N + tn - 1) / tn;
    for (int cm = 0; cm < mt; cm += bm)
      for (int cn = 0; cn < nt; cn += bn)
        for (int im = cm; im < std::min(mt, cm + bm); ++im)
          for (int in = cn; in < std::min(nt, cn + bn); ++in) {
            const int m0 = im * tm, n0 = in * tn;
            const int32_t group = S > 1 ? out.ngroups++ : -1;
            const int32_t slot0 = S > 1 ? out.nslots : -1;
            if (S > 1) out.nslots += static_cast<int32_t>(S);
            for (int64_t sp = 0; sp < S; ++sp) {
              const int64_t s0 = stages * sp / S, s1 = stages * (sp + 1) / S;
              GemmTile t{};
              t.gemm = static_cast<int32_t>(g);
              t.m0 = m0;
              t.n0 = n0;
              t.k0 = static_cast<int32_t>(s0 * BK);
              t.k1 = static_cast<int32_t>(std::min<int64_t>(s1 * BK, d.K));
              t.nsplit = static_cast<int32_t>(S);
              t.split = static_cast<int32_t>(sp);
              t.group = group;
              t.slot0 = slot0;
              if (S > 1 && sp == 0) out.groups.push_back(t);
              // cost in quarter 16-deep stages: MFMA work scaled by the
              // tile's activity, plus prologue/epilogue (~3 stages)
              const double act = tile_activity(tm, tn, d.M - m0, d.N - n0);
              const int64_t cost = static_cast<int64_t>(4.0 * (s1 - s0) * (BK / 16) * act) + 12;
              units.push_back({t, cost});
            }
          }
  }
  return units;
}

// LPT (longest unit first, to the least loaded workgroup) over the
// workgroups taken in the order given, ties going to the earlier one.  The
// order fills one workgroup slot of every CU before the next slot, and
// within a slot walks the CUs of one XCD before the next XCD (workgroup w
// runs on XCD w % kNumXcd, and resident workgroups of an XCD spread over its
// CUs in turn).  So the most expensive units land on distinct CUs (the
// workgroups of a CU share its matrix cores), and runs of consecutive units,
// which come from one cluster, share an XCD.
Sched lpt(const std::vector<GemmDesc>& descs, int tm, int tn, int BK, int num_cu, int bpc, int64_t split_target,
          bool one_per_wg) {
  Sched out;
  const int cpx = std::max(1, num_cu / kNumXcd);
  const int bm = std::max(1, static_cast<int>(std::sqrt(double(cpx))));
  const int bn = std::max(1, cpx / bm);
  std::vector<Unit> units = make_units(descs, tm, tn, BK, split_target, bm, bn, out);
  const int nwg = static_cast<int>(std::min<int64_t>(int64_t(num_cu) * bpc, static_cast<int64_t>(units.size())));
  std::vector<int> order;
  for (int slot = 0; slot < bpc; ++slot)
    for (int x = 0; x < kNumXcd; ++x)
      for (int c = 0; c < cpx; ++c) {
        const int w = x + kNumXcd * (c + cpx * slot);
        if (w < nwg) order.push_back(w);
      }
  for (int w = kNumXcd * cpx * bpc; w < nwg; ++w) order.push_back(w);  // CU counts not a multiple of 8
  std::stable_sort(units.begin(), units.end(), [](const Unit& a, const Unit& b) { return a.cost > b.cost; });
  std::vector<std::vector<GemmTile>> per(nwg);
  std::vector<std::vector<GemmTile>> per_xcd(kNumXcd);  // units in the order dealt, by XCD
  using E = std::pair<int64_t, int>;  // (load, rank in order)
  std::priority_queue<E, std::vector<E>, std::greater<E>> heap;
  for (int v = 0; v < static_cast<int>(order.size()); ++v) heap.push({0, v});
  int64_t mk = 0;
  for (const auto& u : units) {
    E e = heap.top();
    heap.pop();
    per[order[e.second]].push_back(u.t);
    per_xcd[order[e.second] % kNumXcd].push_back(u.t);
    mk = std::max(mk, e.first + u.cost);
    heap.push({e.first + u.cost, e.second});
  }
  // the reduce kernel reads and writes every partial once: at ~5 TB/s one
  // 16-deep fp64 stage of MFMA work (4096 cycles at 2.4 GHz) moves ~8.5 MB
  const double red_bytes = 2.0 * out.nslots * double(tm) * tn * 8.0;
  out.makespan = static_cast<double>(mk) / 4.0 + (out.nslots ? 2.0 + red_bytes / 8.5e6 : 0.0);
  out.wg_first.assign(1, 0);
  if (one_per_wg) {
    // one unit per workgroup, workgroup p taking the next unit the LPT dealt
    // to XCD p % kNumXcd: the hardware starts a new workgroup on a CU as
    // soon as one retires, which balances the CUs of an XCD at run time
    std::vector<size_t> next(kNumXcd, 0);
    for (size_t left = units.size(); left > 0;)
      for (int x = 0; x < kNumXcd; ++x)
        if (next[x] < per_xcd[x].size()) {
          out.tiles.push_back(per_xcd[x][next[x]++]);
          out.wg_first.push_back(static_cast<int32_t>(out.tiles.size()));
          --left;
        }
    return out;
  }
  for (int w = 0; w < nwg; ++w) {
    out.tiles.insert(out.tiles.end(), per[w].begin(), per[w].end());
    out.wg_first.push_back(static_cast<int32_t>(out.tiles.size()));
  }
  return out;
}

// Split-BF16x3 GEMMs run one tile per workgroup: the hardware balancing
// gains that kernel more than the prefetch across tile boundaries of a
// persistent workgroup (its GEMM stage 5-6 % faster on the H_eff D = 4096
// contractions).  The fp64 and fp32 kernels keep persistent workgroups (one
// tile per workgroup was no faster in fp64 and 20 % slower on the split-K
// contraction in fp32).
Sched schedule_tiles(const std::vector<GemmDesc>& descs, int tm, int tn, int tk, int num_cu, int bpc,
                     int precision) {
  const bool one = precision == TK_PREC_BF16X3;
  Sched best = lpt(descs, tm, tn, tk, num_cu, bpc, 0, one);
  if (descs.empty()) return best;
  const int64_t max_wg = int64_t(num_cu) * bpc;
  int64_t total = 0;
  for (const auto& d : descs) total += ((d.M + tm - 1) / tm) * ((d.N + tn - 1) / tn) * ((d.K + tk - 1) / tk);
  for (int per_wg : {2, 3, 4, 6, 8}) {
    const int64_t target = std::max<int64_t>(4, total / (max_wg * per_wg));
    Sched s = lpt(descs, tm, tn, tk, num_cu, bpc, target, one);
    if (s.makespan < 0.97 * best.makespan) best = std::move(s);
  }
  return best;
}

void upload_schedule(DevBuf& d_tiles, DevBuf& d_wg, DevBuf& d_partials, DevBuf& d_groups, const Sched& sc, int tm,
                     int tn) {
  d_tiles.upload(sc.tiles);
  d_wg.upload(sc.wg_first);
  d_partials.alloc(static_cast<size_t>(sc.nslots) * tm * tn * sizeof(double));
  d_groups.upload(sc.groups);
}

void plan_reschedule(tk_plan& P, int tm, int tn, int tk, bool upload = true) {
  P.tile_m = tm;
  P.tile_n = tn;
  P.tile_k = tk;
  const int per_cu = P.ctx ? tk::gemm_blocks_per_cu(P.dtype, P.precision, tm, tn, tk) : 1;
  Sched sc = schedule_tiles(P.descs, tm, tn, tk, P.ctx ? P.ctx->num_cu : 256, per_cu, P.precision);
  P.tiles = sc.tiles;
  P.wg_first = sc.wg_first;
  P.groups = sc.groups;
  P.ngroups = sc.ngroups;
  P.nslots = sc.nslots;
  P.makespan = sc.makespan;
  if (P.ctx && upload) upload_schedule(P.d_tiles, P.d_wg, P.d_partials, P.d_groups, sc, tm, tn);
}

void choose_default_tile(const std::vector<GemmDesc>& descs, int precision, int* tm, int* tn, int* tk) {
  int64_t mmax = 0, nmax = 0, kmax = 0;
  for (const auto& d : descs) {
    mmax = std::max<int64_t>(mmax, d.M);
    nmax = std::max<int64_t>(nmax, d.N);
    kmax = std::max<int64_t>(kmax, d.K);
  }
  *tm = mmax > 64 ? 128 : 64;
  *tn = nmax > 64 ? 128 : 64;
  *tk = (kmax >= 256 || precision == TK_PREC_BF16X3) ? 32 : 16;
}

std::unique_ptr<tk_plan> build_contract_plan(tk_context* ctx, const tk_tensor* A, std::vector<int> pA,
                                             std::vector<int> qA, const tk_tensor* B, std::vector<int> pB,
                                             std::vector<int> qB, std::vector<int> pAB, std::vector<int> qAB,
                                             int precision, const tk_tensor* C) {
  const Structure& sA = *A->st;
  const Structure& sB = *B->st;
  if (sA.sym != sB.sym || sA.sym != C->st->sym) fail(TK_ERR_INVALID_ARG, "symmetry mismatch");
  if (A->dtype != B->dtype || A->dtype != C->dtype) fail(TK_ERR_DTYPE, "dtype mismatch");
  check_perm(pA, qA, sA.N());
  check_perm(pB, qB, sB.N());
  if (qA.size() != pB.size()) fail(TK_ERR_INVALID_ARG, "qA and pB differ in length");
  check_perm(pAB, qAB, static_cast<int>(pA.size() + qB.size()));
  if (precision < TK_PREC_NATIVE || precision > TK_PREC_BF16X3) fail(TK_ERR_INVALID_ARG, "unknown precision");
  if (!tk::gemm_tile_supported(A->dtype, precision, 128, 128, 32))
    fail(TK_ERR_DTYPE, "this dtype / precision combination is not available");

  auto P = std::make_unique<tk_plan>();
  P->ctx = ctx;
  P->A = A->st;
  P->B = B->st;
  P->C = C->st;
  P->pA = pA;
  P->qA = qA;
  P->pB = pB;
  P->qB = qB;
  P->pAB = pAB;
  P->qAB = qAB;
  P->precision = precision;
  P->dtype = A->dtype;
  const int sym = sA.sym;

  std::vector<Space> atc, atd, btc, btd;
  permute_spaces(sA, pA, qA, atc, atd);
  permute_spaces(sB, pB, qB, btc, btd);
  if (atd.size() != btc.size()) fail(TK_ERR_SPACE_MISMATCH, "domain(A~) != codomain(B~)");
  for (size_t k = 0; k < atd.size(); ++k)
    if (atd[k] != btc[k]) fail(TK_ERR_SPACE_MISMATCH, "domain(A~) != codomain(B~) at contracted leg " + std::to_string(k));
  P->At = get_structure(sym, atc, atd);
  P->Bt = get_structure(sym, btc, btd);
  P->Ct = get_structure(sym, atc, btd);
  const Structure& At = *P->At;
  const Structure& Bt = *P->Bt;
  const Structure& Ct = *P->Ct;
  std::vector<Space> cc, cd;
  permute_spaces(Ct, pAB, qAB, cc, cd);
  if (cc != C->st->cod || cd != C->st->dom) fail(TK_ERR_SPACE_MISMATCH, "C does not have the contracted spaces");
  const Structure& sC = *C->st;

  // composition twist: contracted legs on dual spaces (codomain of B~)
  bool twist = false;
  if (sA.si.fermionic)
    for (const auto& s : btc)
      if (s.dual && std::find(s.p.begin(), s.p.end(), 1) != s.p.end()) twist = true;
  P->permA = !is_identity(pA, qA, sA.N1());
  P->permB = !is_identity(pB, qB, sB.N1()) || twist;
  // split-BF16x3: the operands of the MFMA sector GEMMs (K > kSmallK) are
  // written once, by the operand permute, as bf16 hi / lo planes with k
  // contiguous (identity permutations included); small-K sectors keep the
  // element type in the ordinary workspaces
  const bool split = precision == TK_PREC_BF16X3;
  PlaneMap pmA, pmB;
  bool smallk_any = false;
  if (split) {
    pmA.rows = true;
    pmA.buf = tk::kBufAp;
    pmB.buf = tk::kBufBp;
    pmA.off.assign(At.keys.size(), -1);
    pmA.ld.assign(At.keys.size(), 0);
    pmB.off.assign(Bt.keys.size(), -1);
    pmB.ld.assign(Bt.keys.size(), 0);
    for (size_t sa = 0; sa < At.keys.size(); ++sa) {
      const int sb = Bt.sector_of_key(At.keys[sa]);
      if (sb < 0) continue;
      const int64_t K = At.C[sa];
      if (K <= kSmallK) {
        smallk_any = true;
        continue;
      }
      const int64_t ld = (K + 7) / 8 * 8;
      if (ld >= (int64_t(1) << 22))
        fail(TK_ERR_UNSUPPORTED, "split-BF16x3: contracted dimension of one coupled sector above 2^22");
      pmA.off[sa] = P->planeA;
      pmA.ld[sa] = ld;
      P->planeA += At.R[sa] * ld;
      pmB.off[sb] = P->planeB;
      pmB.ld[sb] = ld;
      P->planeB += Bt.C[sb] * ld;
    }
    if (P->planeA > INT32_MAX || P->planeB > INT32_MAX) fail(TK_ERR_UNSUPPORTED, "split-BF16x3 planes above 2^31 elements");
    pmA.lo = static_cast<int32_t>(P->planeA);
    pmB.lo = static_cast<int32_t>(P->planeB);
    P->needA = P->permA && smallk_any;
    P->needB = P->permB && smallk_any;
    plan_permute_tasks(sA, pA, qA, At, tk::kBufA, P->needA ? tk::kBufAt : int16_t(-1), false, P->preA, nullptr,
                       nullptr, &pmA);
    plan_permute_tasks(sB, pB, qB, Bt, tk::kBufB, P->needB ? tk::kBufBt : int16_t(-1), twist, P->preB, nullptr,
                       nullptr, &pmB);
    plan_plane_padding(At, pmA, P->preA);
    plan_plane_padding(Bt, pmB, P->preB);
  } else {
    P->needA = P->permA;
    P->needB = P->permB;
    if (P->permA) plan_permute_tasks(sA, pA, qA, At, tk::kBufA, tk::kBufAt, false, P->preA);
    if (P->permB) plan_permute_tasks(sB, pB, qB, Bt, tk::kBufB, tk::kBufBt, twist, P->preB);
  }
  // the whole operand permute as one list (one launch of each kernel); the
  // per-operand lists are kept apart only when both operands have work, so
  // that either can be enqueued alone (TK_STAGE_PERMUTE_A / _B)
  auto has_work = [](const TaskList& t) { return !t.tasks.empty() || !t.tiles.empty(); };
  P->pre_owner = (has_work(P->preA) ? 1 : 0) | (has_work(P->preB) ? 2 : 0);
  P->pre.tasks = P->preA.tasks;
  P->pre.tasks.insert(P->pre.tasks.end(), P->preB.tasks.begin(), P->preB.tasks.end());
  P->pre.tiles = P->preA.tiles;
  P->pre.tiles.insert(P->pre.tiles.end(), P->preB.tiles.begin(), P->preB.tiles.end());
  pack_workgroups(P->pre);
  if (P->pre_owner == 3) {
    pack_workgroups(P->preA);
    pack_workgroups(P->preB);
  } else {
    for (TaskList* t : {&P->preA, &P->preB}) {
      t->tasks.clear();
      t->tiles.clear();
      t->wg_first.assign(1, 0);
    }
  }

  const bool idC = is_identity(pAB, qAB, Ct.N1());
  // fused scatter needs <= 4 legs per side of C~ and 16-bit leg indices
  bool can_scatter = Ct.N1() <= 4 && Ct.N2() <= 4;
  for (int l = 0; l < Ct.N() && can_scatter; ++l)
    for (int64_t d : Ct.leg(l).deg)
      if (d > 65535) can_scatter = false;
  P->scatter = !idC && can_scatter;
  P->post = !idC && !can_scatter;

  const int16_t abuf = P->permA ? tk::kBufAt : tk::kBufA;
  const int16_t bbuf = P->permB ? tk::kBufBt : tk::kBufB;
  std::vector<int> src(pAB);
  src.insert(src.end(), qAB.begin(), qAB.end());
  std::vector<int> pos(Ct.N());
  for (int n = 0; n < Ct.N(); ++n) pos[src[n]] = n;
  const auto outpairs = sA.si.fermionic ? exchanged_pairs(Ct.N1(), Ct.N2(), pAB, qAB) : std::vector<std::pair<int, int>>{};

  std::vector<uint8_t> tup(Ct.N()), otup(Ct.N());
  int64_t odim[TK_MAX_RANK], ostr[TK_MAX_RANK];
  for (size_t s = 0; s < Ct.keys.size(); ++s) {
    const int64_t key = Ct.keys[s];
    const int sa = At.sector_of_key(key);
    const int64_t M = Ct.R[s], N = Ct.C[s];
    const int64_t K = sa >= 0 ? At.C[sa] : 0;
    const Group& rg = *Ct.rg[s];
    const Group& cg = *Ct.cg[s];
    if (K > 0) {
      const int sb = Bt.sector_of_key(key);
      if (sb < 0) fail(TK_ERR_SPACE_MISMATCH, "internal: B~ lacks a sector of A~");
      GemmDesc d{};
      d.a = At.soff[sa];
      d.b = Bt.soff[sb];
      d.M = checked_i32(M, "M");
      d.N = checked_i32(N, "N");
      d.K = checked_i32(K, "K");
      d.lda = d.M;
      d.ldb = d.K;
      // the GEMM kernels address one stage of A (up to 32 rows of M) and of B
      // (up to 128 columns of K) with 32-bit byte offsets
      if (K > kSmallK && (M >= (int64_t(1) << 23) || K >= (int64_t(1) << 21)))
        fail(TK_ERR_UNSUPPORTED, "MFMA sector GEMM with M >= 2^23 or K >= 2^21");
      d.a_buf = abuf;
      d.b_buf = bbuf;
      P->flops += 2.0 * double(M) * double(N) * double(K);
      P->mnk.insert(P->mnk.end(), {M, N, K});
      if (K <= kSmallK) {
        // row-stationary stream (one thread per row of A~, all columns):
        // channel tables, the output placement of every channel pair, and
        // tasks of up to 256 rows x kSkCols columns.  Outputs go straight
        // to C (identity or fused permute) or, when the output permute runs
        // afterwards, to C~ in its own layout.
        // with the fused scatter (at most 4 legs per side) a channel is
        // decomposed into its legs; in C~'s own layout the position inside
        // a channel is the channel-local index itself (one merged leg)
        const int nrleg = P->scatter ? Ct.N1() : 1, ncleg = P->scatter ? Ct.N2() : 1;
        const int32_t rbase = checked_i32(static_cast<int64_t>(P->skchans.size()), "channel table");
        for (int32_t i = 0; i < rg.n(); ++i) {
          tk::SkChan c{};
          c.off = checked_i32(rg.off[i], "row");
          c.count = checked_i32(rg.size[i], "row");
          for (int l = 0; l < 4; ++l) {
            c.dim[l] = !P->scatter ? (l == 0 ? c.count : 1)
                       : l < Ct.N1() ? checked_i32(Ct.cod[l].deg[rg.idx[size_t(i) * Ct.N1() + l]], "dim")
                                     : 1;
            division_magic(static_cast<uint32_t>(c.dim[l]), &c.mag[l], &c.shr[l]);
          }
          P->skchans.push_back(c);
        }
        const int32_t cbase = checked_i32(static_cast<int64_t>(P->skchans.size()), "channel table");
        for (int32_t j = 0; j < cg.n(); ++j) {
          tk::SkChan c{};
          c.off = checked_i32(cg.off[j], "column");
          c.count = checked_i32(cg.size[j], "column");
          for (int l = 0; l < 4; ++l) {
            c.dim[l] = !P->scatter ? (l == 0 ? c.count : 1)
                       : l < Ct.N2() ? checked_i32(Ct.dom[l].deg[cg.idx[size_t(j) * Ct.N2() + l]], "dim")
                                     : 1;
            division_magic(static_cast<uint32_t>(c.dim[l]), &c.mag[l], &c.shr[l]);
          }
          P->skchans.push_back(c);
        }
        const int32_t pbase = checked_i32(static_cast<int64_t>(P->skpairs.size()), "pair table");
        int64_t cbase_elem = 0;
        if (idC) cbase_elem = sC.soff[sC.sector_of_key(key)];
        else if (P->post) cbase_elem = Ct.soff[s];
        for (int32_t i = 0; i < rg.n(); ++i)
          for (int32_t j = 0; j < cg.n(); ++j) {
            PairDesc pd{};
            pd.sign = 1.0f;
            if (P->scatter) {
              std::copy(rg.idx.begin() + size_t(i) * Ct.N1(), rg.idx.begin() + size_t(i + 1) * Ct.N1(), tup.begin());
              std::copy(cg.idx.begin() + size_t(j) * Ct.N2(), cg.idx.begin() + size_t(j + 1) * Ct.N2(),
                        tup.begin() + Ct.N1());
              for (int n = 0; n < Ct.N(); ++n) otup[n] = tup[src[n]];
              const BlockLoc bl = locate(sC, otup.data());
              if (bl.sector < 0) fail(TK_ERR_SPACE_MISMATCH, "internal: C lacks a channel of C~");
              block_strides(sC, otup.data(), bl.R, odim, ostr);
              pd.base = bl.offset;
              if (sA.si.fermionic && channel_parity(Ct, tup.data(), outpairs)) pd.sign = -1.0f;
              for (int l = 0; l < Ct.N1(); ++l) pd.S[l] = checked_i32(ostr[pos[l]], "stride");
              for (int l = 0; l < Ct.N2(); ++l) pd.S[4 + l] = checked_i32(ostr[pos[Ct.N1() + l]], "stride");
            } else {
              // C~ layout: column-major M x N sector, channels in order
              pd.base = cbase_elem + rg.off[i] + cg.off[j] * M;
              pd.S[0] = 1;
              pd.S[4] = checked_i32(M, "stride");
            }
            P->skpairs.push_back(pd);
          }
        const int16_t dbuf = P->post ? tk::kBufCt : tk::kBufC;
        if (N > kSkCols && dbuf == tk::kBufC &&
            add_output_runs(P->skruns[K], Ct, rg, cg, P->skchans, rbase, cbase, P->skpairs, pbase, src, P->scatter,
                            At.soff[sa], Bt.soff[sb], M, K, abuf, bbuf))
          continue;
        if (N > kSkCols) {
          // many columns: output-stationary tasks over each output block, in
          // the output's leg order (A~ and B~ of such a sector are re-read
          // from cache; the output is written once, in order)
          uint32_t order = 0;
          int nout = 0;
          if (P->scatter) {
            for (int n = 0; n < Ct.N(); ++n) order |= static_cast<uint32_t>(src[n]) << (4 * n);
            nout = Ct.N();
          } else {
            order = 0u | (1u << 4);
            nout = 2;
          }
          auto make = [&](int32_t i, int32_t j) {
            tk::SkBlockTask t{};
            t.a = At.soff[sa] + rg.off[i];
            t.b = Bt.soff[sb];  // the column channel's first column is added per block
            t.lda = d.M;
            t.ldb = d.K;
            t.rchan = rbase + i;
            t.cchan = cbase + j;
            t.pair = pbase + i * cg.n() + j;
            t.order = order;
            t.nrleg = static_cast<int16_t>(nrleg);
            t.ncleg = static_cast<int16_t>(ncleg);
            t.nout = static_cast<int16_t>(nout);
            t.a_buf = abuf;
            t.b_buf = bbuf;
            t.dst_buf = dbuf;
            t.nblk = 1;
            return t;
          };
          // strips of whole blocks of one row channel (consecutive column
          // channels, up to kSkStrip elements); a larger block alone, in
          // chunks
          for (int32_t i = 0; i < rg.n(); ++i)
            for (int32_t j = 0; j < cg.n();) {
              const int64_t blk = rg.size[i] * cg.size[j];
              if (blk > INT32_MAX) fail(TK_ERR_UNSUPPORTED, "block larger than 2^31 elements");
              if (blk > kSkStrip) {
                for (int64_t s0 = 0; s0 < blk; s0 += tk::kPermChunk) {
                  tk::SkBlockTask t = make(i, j);
                  t.start = static_cast<int32_t>(s0);
                  t.count = static_cast<int32_t>(std::min<int64_t>(tk::kPermChunk, blk - s0));
                  P->skblocks[K].tasks.push_back(t);
                }
                ++j;
                continue;
              }
              tk::SkBlockTask t = make(i, j);
              int64_t tot = 0;
              int32_t n = 0;
              while (j < cg.n() && rg.size[i] * cg.size[j] <= kSkStrip && tot + rg.size[i] * cg.size[j] <= kSkStrip) {
                tot += rg.size[i] * cg.size[j];
                ++j;
                ++n;
              }
              t.start = 0;
              t.count = static_cast<int32_t>(tot);
              t.nblk = n;
              P->skblocks[K].tasks.push_back(t);
            }
          continue;
        }
        const int64_t task_rows = int64_t(tk::kThreads) * tk::smallk_rows_per_thread(static_cast<int>(K));
        for (int32_t i = 0; i < rg.n(); ++i)
          for (int64_t r0 = 0; r0 < rg.size[i]; r0 += task_rows)
            for (int64_t n0 = 0, j = 0; n0 < N; n0 += kSkCols) {
              while (cg.off[j] + cg.size[j] <= n0) ++j;
              tk::SmallKTask t{};
              t.a = At.soff[sa] + rg.off[i] + r0;
              t.b = Bt.soff[sb];
              t.lda = d.M;
              t.ldb = d.K;
              t.rows = static_cast<int32_t>(std::min<int64_t>(task_rows, rg.size[i] - r0));
              t.r0 = static_cast<int32_t>(r0);
              t.rchan = rbase + i;
              t.cchan = cbase + static_cast<int32_t>(j);
              t.c0 = static_cast<int32_t>(n0 - cg.off[j]);
              t.ncols = static_cast<int32_t>(std::min<int64_t>(kSkCols, N - n0));
              t.bcol = static_cast<int32_t>(n0);
              t.pair = pbase + i * cg.n() + static_cast<int32_t>(j);
              t.nrleg = static_cast<int16_t>(nrleg);
              t.ncleg = static_cast<int16_t>(ncleg);
              t.a_buf = abuf;
              t.b_buf = bbuf;
              t.dst_buf = dbuf;
              P->smallk[K].tasks.push_back(t);
            }
        continue;
      }
      if (split) {
        d.a = pmA.off[sa];
        d.lda = checked_i32(pmA.ld[sa], "lda");
        d.a_buf = tk::kBufAp;
        d.alo = P->planeA;
        d.b = pmB.off[sb];
        d.ldb = checked_i32(pmB.ld[sb], "ldb");
        d.b_buf = tk::kBufBp;
        d.blo = P->planeB;
      }
      if (idC) {
        d.mode = 0;
        d.c = sC.soff[sC.sector_of_key(key)];
        d.ldc = d.M;
        d.c_buf = tk::kBufC;
      } else if (P->post) {
        d.mode = 0;
        d.c = Ct.soff[s];
        d.ldc = d.M;
        d.c_buf = tk::kBufCt;
      } else {
        d.mode = 1;
        d.c_buf = tk::kBufC;
        d.row_map = checked_i32(static_cast<int64_t>(P->row_map.size()), "row map");
        d.col_map = checked_i32(static_cast<int64_t>(P->col_map.size()), "col map");
        d.pair_base = checked_i32(static_cast<int64_t>(P->pairs.size()), "pair table");
        d.ncc = cg.n();
        // row maps: every row of the sector -> (channel, leg indices)
        for (int32_t i = 0; i < rg.n(); ++i) {
          const uint8_t* t = rg.idx.data() + size_t(i) * Ct.N1();
          for (int64_t r = 0; r < rg.size[i]; ++r) {
            LegMap lm{};
            lm.chan = i;
            int64_t rem = r;
            for (int l = 0; l < Ct.N1(); ++l) {
              const int64_t dl = Ct.cod[l].deg[t[l]];
              lm.idx[l] = static_cast<uint16_t>(rem % dl);
              rem /= dl;
            }
            P->row_map.push_back(lm);
          }
        }
        for (int32_t j = 0; j < cg.n(); ++j) {
          const uint8_t* t = cg.idx.data() + size_t(j) * Ct.N2();
          for (int64_t c = 0; c < cg.size[j]; ++c) {
            LegMap lm{};
            lm.chan = j;
            int64_t rem = c;
            for (int l = 0; l < Ct.N2(); ++l) {
              const int64_t dl = Ct.dom[l].deg[t[l]];
              lm.idx[l] = static_cast<uint16_t>(rem % dl);
              rem /= dl;
            }
            P->col_map.push_back(lm);
          }
        }
        for (int32_t i = 0; i < rg.n(); ++i) {
          for (int32_t j = 0; j < cg.n(); ++j) {
            std::copy(rg.idx.begin() + size_t(i) * Ct.N1(), rg.idx.begin() + size_t(i + 1) * Ct.N1(), tup.begin());
            std::copy(cg.idx.begin() + size_t(j) * Ct.N2(), cg.idx.begin() + size_t(j + 1) * Ct.N2(),
                      tup.begin() + Ct.N1());
            for (int n = 0; n < Ct.N(); ++n) otup[n] = tup[src[n]];
            const BlockLoc b = locate(sC, otup.data());
            if (b.sector < 0) fail(TK_ERR_SPACE_MISMATCH, "internal: C lacks a channel of C~");
            block_strides(sC, otup.data(), b.R, odim, ostr);
            PairDesc pd{};
            pd.base = b.offset;
            const int par = sA.si.fermionic ? channel_parity(Ct, tup.data(), outpairs) : 0;
            pd.sign = par ? -1.0f : 1.0f;
            for (int l = 0; l < Ct.N1(); ++l) pd.S[l] = checked_i32(ostr[pos[l]], "stride");
            for (int l = 0; l < Ct.N2(); ++l) pd.S[4 + l] = checked_i32(ostr[pos[Ct.N1() + l]], "stride");
            P->pairs.push_back(pd);
          }
        }
      }
      P->descs.push_back(d);
    } else {
      // empty K range: the C~ block is zero (eq. abelian_compostion remark)
      ++P->nzero;
      if (idC) {
        const int sc = sC.sector_of_key(key);
        P->zranges.add(tk::kBufC, sC.soff[sc], M * N);
      } else if (P->post) {
        P->zranges.add(tk::kBufCt, Ct.soff[s], M * N);
      } else {
        for (int32_t j = 0; j < cg.n(); ++j)
          for (int32_t i = 0; i < rg.n(); ++i) {
            std::copy(rg.idx.begin() + size_t(i) * Ct.N1(), rg.idx.begin() + size_t(i + 1) * Ct.N1(), tup.begin());
            std::copy(cg.idx.begin() + size_t(j) * Ct.N2(), cg.idx.begin() + size_t(j + 1) * Ct.N2(),
                      tup.begin() + Ct.N1());
            for (int n = 0; n < Ct.N(); ++n) otup[n] = tup[src[n]];
            const BlockLoc b = locate(sC, otup.data());
            if (b.sector < 0) fail(TK_ERR_SPACE_MISMATCH, "internal: C lacks a channel of C~");
            block_strides(sC, otup.data(), b.R, odim, ostr);
            int64_t span = 0;
            if (contiguous_block(sC.N(), odim, ostr, &span)) {
              P->zranges.add(tk::kBufC, b.offset, span);
            } else {
              int64_t zs[TK_MAX_RANK] = {0};
              add_block_tasks(P->zero, -1, 0, tk::kBufC, b.offset, sC.N(), odim, zs, ostr, 1.0f);
            }
          }
      }
    }
  }
  P->zranges.finalize();
  for (auto& r : P->skruns) r.finalize();
  pack_workgroups(P->zero);
  for (auto& l : P->skblocks) pack_workgroups(l);
  if (P->post) {
    plan_permute_tasks(Ct, pAB, qAB, sC, tk::kBufCt, tk::kBufC, false, P->postp);
    pack_workgroups(P->postp);
  }

  int tm, tn, tkk;
  choose_default_tile(P->descs, precision, &tm, &tn, &tkk);
  plan_reschedule(*P, tm, tn, tkk, false);  // uploads follow below

  if (ctx) {
    const size_t es = A->esize();
    if (P->needA) P->wsA.alloc(At.size * es);
    if (P->needB) P->wsB.alloc(Bt.size * es);
    if (P->post) P->wsC.alloc(Ct.size * es);
    if (P->planeA) P->wsAp.alloc(4 * P->planeA);  // two bf16 planes
    if (P->planeB) P->wsBp.alloc(4 * P->planeB);
    P->pre.upload();
    P->preA.upload();
    P->preB.upload();
    P->zero.upload();
    P->zranges.upload();
    P->postp.upload();
    P->d_descs.upload(P->descs);
    P->d_rowmap.upload(P->row_map);
    P->d_colmap.upload(P->col_map);
    P->d_pairs.upload(P->pairs);
    for (auto& l : P->smallk) l.upload();
    for (auto& l : P->skblocks) l.upload();
    for (auto& r : P->skruns) r.upload();
    P->d_skchans.upload(P->skchans);
    P->d_skpairs.upload(P->skpairs);
    Sched sc;
    sc.tiles = P->tiles;
    sc.wg_first = P->wg_first;
    sc.groups = P->groups;
    sc.ngroups = P->ngroups;
    sc.nslots = P->nslots;
    upload_schedule(P->d_tiles, P->d_wg, P->d_partials, P->d_groups, sc, P->tile_m, P->tile_n);
  }
  return P;
}

tk::Ptrs plan_ptrs(const tk_plan& P, const tk_tensor* A, const tk_tensor* B, tk_tensor* C) {
  tk::Ptrs p{};
  p.p[tk::kBufA] = A->data;
  p.p[tk::kBufB] = B->data;
  p.p[tk::kBufC] = C->data;
  p.p[tk::kBufAt] = P.wsA.p;
  p.p[tk::kBufBt] = P.wsB.p;
  p.p[tk::kBufCt] = P.wsC.p;
  p.p[tk::kBufAp] = P.wsAp.p;
  p.p[tk::kBufBp] = P.wsBp.p;
  p.table = nullptr;
  return p;
}

void check_exec_tensor(const tk_tensor* t, const std::shared_ptr<Structure>& st, int dtype, const char* what) {
  if (!t) fail(TK_ERR_INVALID_ARG, std::string("null tensor ") + what);
  if (!t->data && t->st->size > 0) fail(TK_ERR_INVALID_ARG, std::string("tensor without data: ") + what);
  if (t->st != st && t->st->sig != st->sig) fail(TK_ERR_SPACE_MISMATCH, std::string("structure differs from the plan: ") + what);
  if (t->dtype != dtype) fail(TK_ERR_DTYPE, std::string("dtype differs from the plan: ") + what);
}

void execute_plan(tk_plan& P, const tk_tensor* A, const tk_tensor* B, tk_tensor* C, double alpha, double beta,
                  hipStream_t stream, int stages = TK_STAGE_ALL) {
  if (!P.ctx) fail(TK_ERR_INVALID_ARG, "plan was made without a context");
  check_exec_tensor(A, P.A, P.dtype, "A");
  check_exec_tensor(B, P.B, P.dtype, "B");
  check_exec_tensor(C, P.C, P.dtype, "C");
  if (C->data && (C->data == A->data || C->data == B->data)) fail(TK_ERR_INVALID_ARG, "C aliases an operand");
  tk::Ptrs ptrs = plan_ptrs(P, A, B, C);
  {
    const bool pa = (stages & (TK_STAGE_PERMUTE | TK_STAGE_PERMUTE_A)) != 0;
    const bool pb = (stages & (TK_STAGE_PERMUTE | TK_STAGE_PERMUTE_B)) != 0;
    const bool split = P.precision == TK_PREC_BF16X3;
    // one operand alone: its own list when both have work, else the whole
    // list if it is that operand's
    const TaskList* tl = nullptr;
    if (pa && pb) tl = &P.pre;
    else if (pa) tl = P.pre_owner == 3 ? &P.preA : P.pre_owner == 1 ? &P.pre : nullptr;
    else if (pb) tl = P.pre_owner == 3 ? &P.preB : P.pre_owner == 2 ? &P.pre : nullptr;
    if (tl) launch_tasklist(P.dtype, *tl, ptrs, 1.0, 0.0, stream, split, "permute launch");
  }
  const double ga = alpha, gb = P.post ? 0.0 : beta;
  if ((stages & TK_STAGE_GEMM) && !P.descs.empty()) {
    tk::GemmArgs ga_{};
    ga_.descs = static_cast<const GemmDesc*>(P.d_descs.p);
    ga_.tiles = static_cast<const GemmTile*>(P.d_tiles.p);
    ga_.wg_first = static_cast<const int32_t*>(P.d_wg.p);
    ga_.row_map = static_cast<const LegMap*>(P.d_rowmap.p);
    ga_.col_map = static_cast<const LegMap*>(P.d_colmap.p);
    ga_.pairs = static_cast<const PairDesc*>(P.d_pairs.p);
    ga_.partials = static_cast<double*>(P.d_partials.p);
    ga_.ptrs = ptrs;
    ga_.alpha = P.post ? 1.0 : ga;
    ga_.beta = gb;
    hip_check(tk::launch_gemm(P.dtype, P.precision, P.tile_m, P.tile_n, P.tile_k, ga_,
                              static_cast<int>(P.wg_first.size()) - 1, stream),
              "gemm launch");
    hip_check(tk::launch_splitk_reduce(P.dtype, P.precision, P.tile_m, P.tile_n, P.tile_k, ga_,
                                       static_cast<const GemmTile*>(P.d_groups.p), P.ngroups, stream),
              "split-K reduce launch");
  }
  if (stages & TK_STAGE_GEMM)
    for (int K = 1; K <= kSmallK; ++K)
      if (P.smallk[K].n() > 0)
        hip_check(tk::launch_smallk(P.dtype, P.precision, K, static_cast<const tk::SmallKTask*>(P.smallk[K].d_tasks.p),
                                    P.smallk[K].n(), static_cast<const tk::SkChan*>(P.d_skchans.p),
                                    static_cast<const PairDesc*>(P.d_skpairs.p), ptrs, P.post ? 1.0 : alpha,
                                    P.post ? 0.0 : beta, stream),
                  "small-K launch");
  if (stages & TK_STAGE_GEMM)
    for (int K = 1; K <= kSmallK; ++K)
      if (P.skblocks[K].nwg() > 0)
        hip_check(tk::launch_smallk_blocks(P.dtype, P.precision, K,
                                           static_cast<const tk::SkBlockTask*>(P.skblocks[K].d_tasks.p),
                                           static_cast<const int32_t*>(P.skblocks[K].d_wg.p), P.skblocks[K].nwg(),
                                           static_cast<const tk::SkChan*>(P.d_skchans.p),
                                           static_cast<const PairDesc*>(P.d_skpairs.p), ptrs, P.post ? 1.0 : alpha,
                                           P.post ? 0.0 : beta, stream),
                  "small-K block launch");
  if (stages & TK_STAGE_GEMM)
    for (int K = 1; K <= kSmallK; ++K)
      if (P.skruns[K].nwg() > 0)
        hip_check(tk::launch_smallk_runs(P.dtype, P.precision, K, static_cast<const tk::SkRun*>(P.skruns[K].d_runs.p),
                                         static_cast<int>(P.skruns[K].runs.size()),
                                         static_cast<const int32_t*>(P.skruns[K].d_first.p),
                                         static_cast<const int64_t*>(P.skruns[K].d_wstart.p), P.skruns[K].nwg(),
                                         static_cast<const tk::SkRunShape*>(P.skruns[K].d_shapes.p), ptrs,
                                         P.post ? 1.0 : alpha, P.post ? 0.0 : beta, stream),
                  "small-K run launch");
  if ((stages & TK_STAGE_ZERO) && P.zranges.nwg() > 0)
    hip_check(tk::launch_zero_ranges(P.dtype, static_cast<const tk::ZeroRange*>(P.zranges.d_ranges.p),
                                     static_cast<int>(P.zranges.ranges.size()),
                                     static_cast<const int32_t*>(P.zranges.d_first.p),
                                     static_cast<const int64_t*>(P.zranges.d_wstart.p), P.zranges.nwg(), ptrs, P.post ? 0.0 : beta, stream),
              "zero-range launch");
  if (stages & TK_STAGE_ZERO)
    launch_tasklist(P.dtype, P.zero, ptrs, P.post ? 1.0 : alpha, P.post ? 0.0 : beta, stream, false, "zero launch");
  if ((stages & TK_STAGE_ZERO) && P.post)
    launch_tasklist(P.dtype, P.postp, ptrs, alpha, beta, stream, false, "permute launch");
}

std::string plan_key(const tk_tensor* A, const std::vector<int>& pA, const std::vector<int>& qA, const tk_tensor* B,
                     const std::vector<int>& pB, const std::vector<int>& qB, const std::vector<int>& pAB,
                     const std::vector<int>& qAB, int prec, const tk_tensor* C) {
  auto lst = [](const std::vector<int>& v) {
    std::string s;
    for (int x : v) s += std::to_string(x) + ",";
    return s + "/";
  };
  return A->st->sig + "#" + B->st->sig + "#" + C->st->sig + "#" + lst(pA) + lst(qA) + lst(pB) + lst(qB) + lst(pAB) +
         lst(qAB) + std::to_string(prec) + "/" + std::to_string(A->dtype);
}

std::vector<Space> make_spaces(int sym, const tk_space* s, int32_t n) {
  if (n < 0 || n > TK_MAX_LEGS || (n > 0 && !s)) fail(TK_ERR_INVALID_ARG, "bad space list");
  std::vector<Space> v;
  for (int i = 0; i < n; ++i) v.push_back(make_space(sym, s[i]));
  return v;
}

tk_tensor* new_tensor(tk_context* ctx, std::shared_ptr<Structure> st, int dtype, void* buf, uint64_t bytes) {
  if (dtype != TK_F64 && dtype != TK_F32) fail(TK_ERR_DTYPE, "dtype must be TK_F64 or TK_F32");
  auto t = std::make_unique<tk_tensor>();
  t->ctx = ctx;
  t->st = std::move(st);
  t->dtype = dtype;
  const uint64_t need = static_cast<uint64_t>(t->st->size) * t->esize();
  if (!ctx) {
    if (buf) fail(TK_ERR_INVALID_ARG, "a structure-only tensor takes no buffer");
  } else if (buf) {
    if (bytes < need) fail(TK_ERR_INVALID_ARG, "buffer smaller than the tensor");
    t->data = buf;
    t->bytes = bytes;
  } else if (need > 0) {
    hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    if (hipMalloc(&t->data, need) != hipSuccess) {
      (void)hipGetLastError();
      t->data = nullptr;
      fail(TK_ERR_OOM, "device allocation failed");
    }
    g_device_allocs.fetch_add(1, std::memory_order_relaxed);
    t->bytes = need;
    t->owns = true;
  }
  return t.release();
}

template <typename F>
tk_status guarded(F&& f) {
  try {
    f();
    return TK_OK;
  } catch (const TkError& e) {
    g_err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return TK_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return TK_ERR_INVALID_ARG;
  }
}

// Per-device state of the allocation-free entry point: the address of the
// device's scratch array (looked up once, when the first context on that
// device is created, with the device current), the host staging of the
// tables of the last call, and an event marking that their copy has left
// host memory.  Calls on one device serialise their host side on `mu`; their
// device work shares the one scratch array (see tk.h).
struct Scratch {
  std::mutex mu;
  void* base = nullptr;
  hipEvent_t copied = nullptr;
  bool pending = false;
  std::vector<char> staging;
};
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::array<std::unique_ptr<Scratch>, kMaxDevices> g_scratch;

void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) fail(TK_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch[device]) return;
  auto S = std::make_unique<Scratch>();
  hip_check(tk::scratch_address(&S->base), "hipGetSymbolAddress of the scratch array");
  hip_check(hipEventCreateWithFlags(&S->copied, hipEventDisableTiming), "hipEventCreate");
  g_scratch[device] = std::move(S);
}

Scratch& scratch_of(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices || !g_scratch[device])
    fail(TK_ERR_INVALID_ARG, "no scratch for this device (create a context first)");
  return *g_scratch[device];
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* tk_last_error(void) { return g_err.c_str(); }
const char* tk_version(void) { return "tk 0.1 (gfx950)"; }

tk_status tk_context_create(int32_t device, tk_context** out) {
  return guarded([&] {
    if (!out) fail(TK_ERR_INVALID_ARG, "null out");
    int n = 0;
    hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) fail(TK_ERR_INVALID_ARG, "no such device");
    hip_check(hipSetDevice(device), "hipSetDevice");
    scratch_setup(device);
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    auto c = std::make_unique<tk_context>();
    c->device = device;
    c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    *out = c.release();
  });
}

tk_status tk_context_destroy(tk_context* ctx) {
  return guarded([&] { delete ctx; });
}

tk_status tk_tensor_create(tk_context* ctx, int32_t sym, int32_t dtype, const tk_space* cod, int32_t ncod,
                           const tk_space* dom, int32_t ndom, void* device_buf, uint64_t buf_bytes, tk_tensor** out) {
  return guarded([&] {
    if (!out) fail(TK_ERR_INVALID_ARG, "null out");
    sym_info(sym);
    auto c = make_spaces(sym, cod, ncod);
    auto d = make_spaces(sym, dom, ndom);
    if (c.size() + d.size() > TK_MAX_RANK) fail(TK_ERR_UNSUPPORTED, "rank above TK_MAX_RANK");
    *out = new_tensor(ctx, get_structure(sym, c, d), dtype, device_buf, buf_bytes);
  });
}

tk_status tk_tensor_destroy(tk_tensor* t) {
  return guarded([&] { delete t; });
}

tk_status tk_tensor_info(const tk_tensor* t, int32_t* sym, int32_t* dtype, int32_t* ncod, int32_t* ndom,
                         int64_t* nelem, int64_t* nblocks, int64_t* nsectors) {
  return guarded([&] {
    if (!t) fail(TK_ERR_INVALID_ARG, "null tensor");
    if (sym) *sym = t->st->sym;
    if (dtype) *dtype = t->dtype;
    if (ncod) *ncod = t->st->N1();
    if (ndom) *ndom = t->st->N2();
    if (nelem) *nelem = t->st->size;
    if (nblocks) *nblocks = t->st->nblocks;
    if (nsectors) *nsectors = static_cast<int64_t>(t->st->keys.size());
  });
}

tk_status tk_tensor_blocks(const tk_tensor* t, int64_t first, int64_t count, int32_t* sector_idx, int64_t* offsets,
                           int64_t* ld) {
  return guarded([&] {
    if (!t) fail(TK_ERR_INVALID_ARG, "null tensor");
    const Structure& st = *t->st;
    if (first < 0 || count < 0 || first + count > st.nblocks) fail(TK_ERR_INVALID_ARG, "block range out of bounds");
    if (count == 0) return;
    int s = static_cast<int>(std::upper_bound(st.bbase.begin(), st.bbase.end(), first) - st.bbase.begin()) - 1;
    for (int64_t b = first; b < first + count; ++b) {
      while (s + 1 < static_cast<int>(st.bbase.size()) && st.bbase[s + 1] <= b) ++s;
      const Group& rg = *st.rg[s];
      const Group& cg = *st.cg[s];
      const int64_t local = b - st.bbase[s];
      const int32_t j = static_cast<int32_t>(local / rg.n()), i = static_cast<int32_t>(local % rg.n());
      const int64_t k = b - first;
      if (sector_idx) {
        for (int l = 0; l < st.N1(); ++l) sector_idx[k * st.N() + l] = rg.idx[size_t(i) * st.N1() + l];
        for (int l = 0; l < st.N2(); ++l) sector_idx[k * st.N() + st.N1() + l] = cg.idx[size_t(j) * st.N2() + l];
      }
      if (offsets) offsets[k] = st.soff[s] + cg.off[j] * st.R[s] + rg.off[i];
      if (ld) ld[k] = st.R[s];
    }
  });
}

tk_status tk_tensor_sectors(const tk_tensor* t, int64_t first, int64_t count, int32_t* charges, int64_t* rows,
                            int64_t* cols, int64_t* offsets) {
  return guarded([&] {
    if (!t) fail(TK_ERR_INVALID_ARG, "null tensor");
    const Structure& st = *t->st;
    const int64_t ns = static_cast<int64_t>(st.keys.size());
    if (first < 0 || count < 0 || first + count > ns) fail(TK_ERR_INVALID_ARG, "sector range out of bounds");
    for (int64_t k = 0; k < count; ++k) {
      const int64_t s = first + k, key = st.keys[s];
      const int64_t p = ((key % 2) + 2) % 2, q = (key - p) / 2;
      if (charges) {
        if (st.sym == TK_SYM_Z2 || st.sym == TK_SYM_FZ2) charges[k] = static_cast<int32_t>(p);
        if (st.sym == TK_SYM_U1) charges[k] = static_cast<int32_t>(q);
        if (st.sym == TK_SYM_U1_FZ2) {
          charges[2 * k] = static_cast<int32_t>(q);
          charges[2 * k + 1] = static_cast<int32_t>(p);
        }
      }
      if (rows) rows[k] = st.R[s];
      if (cols) cols[k] = st.C[s];
      if (offsets) offsets[k] = st.soff[s];
    }
  });
}

tk_status tk_tensor_space(const tk_tensor* t, int32_t leg, tk_space* out) {
  return guarded([&] {
    if (!t || !out) fail(TK_ERR_INVALID_ARG, "null argument");
    if (leg < 0 || leg >= t->st->N()) fail(TK_ERR_INVALID_ARG, "leg out of range");
    const Space& s = t->st->leg(leg);
    out->nsect = s.n();
    out->charges = s.raw.empty() ? nullptr : s.raw.data();
    out->degeneracies = s.deg.data();
    out->isdual = s.dual ? 1 : 0;
  });
}

tk_status tk_tensor_data(const tk_tensor* t, void** device_ptr, uint64_t* bytes) {
  return guarded([&] {
    if (!t) fail(TK_ERR_INVALID_ARG, "null tensor");
    if (device_ptr) *device_ptr = t->data;
    if (bytes) *bytes = static_cast<uint64_t>(t->st->size) * t->esize();
  });
}

tk_status tk_tensor_create_permuted(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np,
                                    const int32_t* q, int32_t nq, void* device_buf, uint64_t buf_bytes,
                                    tk_tensor** out) {
  return guarded([&] {
    if (!A || !out) fail(TK_ERR_INVALID_ARG, "null argument");
    auto pv = to_vec(p, np, "p");
    auto qv = to_vec(q, nq, "q");
    check_perm(pv, qv, A->st->N());
    std::vector<Space> c, d;
    permute_spaces(*A->st, pv, qv, c, d);
    *out = new_tensor(ctx, get_structure(A->st->sym, c, d), A->dtype, device_buf, buf_bytes);
  });
}

tk_status tk_tensor_create_traced(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np,
                                  const int32_t* q, int32_t nq, const int32_t* t1, const int32_t* t2, int32_t nt,
                                  void* device_buf, uint64_t buf_bytes, tk_tensor** out) {
  return guarded([&] {
    if (!A || !out) fail(TK_ERR_INVALID_ARG, "null argument");
    auto pv = to_vec(p, np, "p"), qv = to_vec(q, nq, "q"), a = to_vec(t1, nt, "t1"), b = to_vec(t2, nt, "t2");
    check_trace_lists(*A->st, pv, qv, a, b);
    std::vector<Space> c, d;
    permute_spaces(*A->st, pv, qv, c, d);
    *out = new_tensor(ctx, get_structure(A->st->sym, c, d), A->dtype, device_buf, buf_bytes);
  });
}

tk_status tk_tensor_create_contracted(tk_context* ctx, const tk_tensor* A, const int32_t* pA, int32_t npA,
                                      const int32_t* qA, int32_t nqA, const tk_tensor* B, const int32_t* pB,
                                      int32_t npB, const int32_t* qB, int32_t nqB, const int32_t* pAB, int32_t npAB,
                                      const int32_t* qAB, int32_t nqAB, void* device_buf, uint64_t buf_bytes,
                                      tk_tensor** out) {
  return guarded([&] {
    if (!A || !B || !out) fail(TK_ERR_INVALID_ARG, "null argument");
    if (A->st->sym != B->st->sym) fail(TK_ERR_INVALID_ARG, "symmetry mismatch");
    if (A->dtype != B->dtype) fail(TK_ERR_DTYPE, "dtype mismatch");
    auto pa = to_vec(pA, npA, "pA"), qa = to_vec(qA, nqA, "qA"), pb = to_vec(pB, npB, "pB"), qb = to_vec(qB, nqB, "qB");
    auto pab = to_vec(pAB, npAB, "pAB"), qab = to_vec(qAB, nqAB, "qAB");
    check_perm(pa, qa, A->st->N());
    check_perm(pb, qb, B->st->N());
    if (qa.size() != pb.size()) fail(TK_ERR_INVALID_ARG, "qA and pB differ in length");
    check_perm(pab, qab, static_cast<int>(pa.size() + qb.size()));
    std::vector<Space> atc, atd, btc, btd;
    permute_spaces(*A->st, pa, qa, atc, atd);
    permute_spaces(*B->st, pb, qb, btc, btd);
    for (size_t k = 0; k < atd.size(); ++k)
      if (atd[k] != btc[k]) fail(TK_ERR_SPACE_MISMATCH, "domain(A~) != codomain(B~)");
    Structure tmp;
    tmp.sym = A->st->sym;
    tmp.cod = atc;
    tmp.dom = btd;
    std::vector<Space> c, d;
    permute_spaces(tmp, pab, qab, c, d);
    if (c.size() + d.size() > TK_MAX_RANK || c.size() > TK_MAX_LEGS || d.size() > TK_MAX_LEGS)
      fail(TK_ERR_UNSUPPORTED, "result rank too large");
    *out = new_tensor(ctx, get_structure(A->st->sym, c, d), A->dtype, device_buf, buf_bytes);
  });
}

tk_status tk_tensor_create_adjoint(tk_context* ctx, const tk_tensor* A, void* device_buf, uint64_t buf_bytes,
                                   tk_tensor** out) {
  return guarded([&] {
    if (!A || !out) fail(TK_ERR_INVALID_ARG, "null argument");
    *out = new_tensor(ctx, get_structure(A->st->sym, A->st->dom, A->st->cod), A->dtype, device_buf, buf_bytes);
  });
}

tk_status tk_tensor_permute(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np, const int32_t* q,
                            int32_t nq, tk_tensor* C, void* stream) {
  return guarded([&] {
    if (!ctx || !A || !C) fail(TK_ERR_INVALID_ARG, "null argument");
    if (A->dtype != C->dtype) fail(TK_ERR_DTYPE, "dtype mismatch");
    if (!A->data && A->st->size) fail(TK_ERR_INVALID_ARG, "A has no data");
    if (!C->data && C->st->size) fail(TK_ERR_INVALID_ARG, "C has no data");
    if (A->data && A->data == C->data) fail(TK_ERR_INVALID_ARG, "C aliases A");
    auto pv = to_vec(p, np, "p");
    auto qv = to_vec(q, nq, "q");
    check_perm(pv, qv, A->st->N());
    std::vector<Space> c, d;
    permute_spaces(*A->st, pv, qv, c, d);
    if (c != C->st->cod || d != C->st->dom) fail(TK_ERR_SPACE_MISMATCH, "C does not have the permuted spaces");
    std::string key = "P#" + A->st->sig + "#" + C->st->sig + "#";
    for (int x : pv) key += std::to_string(x) + ",";
    key += "/";
    for (int x : qv) key += std::to_string(x) + ",";
    std::shared_ptr<PermPlan> pp;
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      auto it = ctx->perm_plans.find(key);
      if (it != ctx->perm_plans.end()) pp = it->second;
    }
    if (!pp) {
      pp = std::make_shared<PermPlan>();
      pp->A = A->st;
      pp->C = C->st;
      plan_permute_tasks(*A->st, pv, qv, *C->st, tk::kBufA, tk::kBufC, false, pp->tl);
      pack_workgroups(pp->tl);
      pp->tl.upload();
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->perm_plans[key] = pp;
    }
    tk::Ptrs ptrs{};
    ptrs.p[tk::kBufA] = A->data;
    ptrs.p[tk::kBufC] = C->data;
    launch_tasklist(A->dtype, pp->tl, ptrs, 1.0, 0.0, static_cast<hipStream_t>(stream), false, "permute launch");
  });
}

}  // extern "C"

// Truncated SVD in progress (Alg. "Abelian tensor decomposition"): the
// working copies and singular values on the device, the kept singular
// values per sector, and the structures of the factors.
struct tk_svd {
  tk_context* ctx = nullptr;
  int dtype = TK_F64;
  std::shared_ptr<Structure> T;  // A~ = permute(A, (p, q))
  DevBuf at, ws, secs;           // A~ (when permuted), workspace, sector records
  std::vector<tk::SvdSector> sec;
  std::vector<std::vector<int32_t>> keep;  // per record: kept singular value indices, largest first
  std::vector<int32_t> sec_sector;         // per record: its sector of A~
  std::vector<double> sigma;
  std::shared_ptr<Structure> U, S, V;
  double err = 0.0;
  int max_sweeps = 0;  // largest sweep count over the sectors
};

namespace {
constexpr int kSvdMaxSweeps = 60;
}

namespace {
// The bond space of the factors: one sector per coupled charge with kept
// singular values, that charge as its label.
Space bond_space(const Structure& T, const std::vector<int32_t>& sectors, const std::vector<int64_t>& degs) {
  const SymInfo si = sym_info(T.sym);
  std::vector<int32_t> ch;
  for (int32_t s : sectors) {
    const int64_t key = T.keys[s];
    const int32_t q = static_cast<int32_t>(key >> 1), par = static_cast<int32_t>(key & 1);
    if (T.sym == TK_SYM_U1) ch.push_back(q);
    else if (T.sym == TK_SYM_Z2 || T.sym == TK_SYM_FZ2) ch.push_back(par);
    else if (T.sym == TK_SYM_U1_FZ2) ch.push_back(q), ch.push_back(par);
  }
  tk_space sp{};
  sp.nsect = static_cast<int32_t>(sectors.size());
  sp.charges = si.ncomp ? ch.data() : nullptr;
  sp.degeneracies = degs.data();
  sp.isdual = 0;
  return make_space(T.sym, sp);
}
}  // namespace

extern "C" {

tk_status tk_svd_create(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np, const int32_t* q,
                        int32_t nq, int64_t max_dim, double cutoff, void* stream, tk_svd** out) {
  return guarded([&] {
    if (!ctx || !A || !out) fail(TK_ERR_INVALID_ARG, "null argument");
    if (A->dtype != TK_F64) fail(TK_ERR_DTYPE, "the SVD works on fp64 tensors");
    if (!A->data && A->st->size) fail(TK_ERR_INVALID_ARG, "A has no data");
    auto pv = to_vec(p, np, "p"), qv = to_vec(q, nq, "q");
    check_perm(pv, qv, A->st->N());
    if (pv.empty() || qv.empty()) fail(TK_ERR_INVALID_ARG, "both sides of the matrix form need a leg");
    auto sv = std::make_unique<tk_svd>();
    sv->ctx = ctx;
    std::vector<Space> c, d;
    permute_spaces(*A->st, pv, qv, c, d);
    sv->T = get_structure(A->st->sym, c, d);
    const Structure& T = *sv->T;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double* X = static_cast<const double*>(A->data);
    if (!is_identity(pv, qv, A->st->N1())) {
      sv->at.alloc(T.size * sizeof(double));
      TaskList tl;
      plan_permute_tasks(*A->st, pv, qv, T, tk::kBufA, tk::kBufC, false, tl);
      pack_workgroups(tl);
      tl.upload();
      tk::Ptrs ptrs{};
      ptrs.p[tk::kBufA] = A->data;
      ptrs.p[tk::kBufC] = sv->at.p;
      launch_tasklist(TK_F64, tl, ptrs, 1.0, 0.0, st, false, "permute launch");
      hip_check(hipStreamSynchronize(st), "stream synchronize");  // tl is freed on return
      X = static_cast<const double*>(sv->at.p);
    }
    int64_t wsz = 0;
    for (size_t k = 0; k < T.keys.size(); ++k) {
      const int64_t R = T.R[k], C = T.C[k];
      if (R == 0 || C == 0) continue;
      if (R >= (int64_t(1) << 31) || C >= (int64_t(1) << 31)) fail(TK_ERR_UNSUPPORTED, "sector matrix too large");
      tk::SvdSector r{};
      r.x = T.soff[k];
      r.R = static_cast<int32_t>(R);
      r.C = static_cast<int32_t>(C);
      r.trans = R < C;
      r.m = static_cast<int32_t>(std::max(R, C));
      r.n = static_cast<int32_t>(std::min(R, C));
      r.w = wsz;
      wsz += int64_t(r.m) * r.n;
      r.v = wsz;
      wsz += int64_t(r.n) * r.n;
      sv->sec.push_back(r);
      sv->sec_sector.push_back(static_cast<int32_t>(k));
    }
    for (auto& r : sv->sec) {  // singular values after every matrix
      r.s = wsz;
      wsz += r.n;
    }
    sv->ws.alloc(std::max<int64_t>(wsz, 1) * sizeof(double));
    sv->secs.upload(sv->sec);
    const double tol = std::numeric_limits<double>::epsilon();  // scaled per sector in the kernel
    // Block one-sided Jacobi: the columns of each sector form blocks of
    // kSvdBlock; round g of a sweep holds the g-th round of the round-robin
    // pairing of every sector's blocks (a sector with b blocks has b' - 1
    // rounds, b' = b rounded up to even; one block alone: one round).
    const int nsec = static_cast<int>(sv->sec.size());
    std::vector<std::vector<tk::SvdItem>> rounds;
    for (int r = 0; r < nsec; ++r) {
      const int n = sv->sec[r].n, B = tk::kSvdBlock;
      const int nb = (n + B - 1) / B;
      if (nb <= 1) {
        if (rounds.empty()) rounds.resize(1);
        rounds[0].push_back({r, 0, n, 0, 0, 0});
        continue;
      }
      const int nbp = nb + (nb & 1);
      if (static_cast<int>(rounds.size()) < nbp - 1) rounds.resize(nbp - 1);
      for (int g = 0; g < nbp - 1; ++g)
        for (int i = 0; i < nbp / 2; ++i) {
          const int P = i == 0 ? 0 : 1 + (g + i) % (nbp - 1);
          const int Q = i == 0 ? 1 + g : 1 + (g - i + nbp - 1) % (nbp - 1);
          const int p0 = std::min(n, P * B), np = std::min(n, (P + 1) * B) - p0;
          const int q0 = std::min(n, Q * B), nq = std::min(n, (Q + 1) * B) - q0;
          if (np > 0) rounds[g].push_back({r, p0, np, q0, nq, 0});
          else if (nq > 0) rounds[g].push_back({r, q0, nq, 0, 0, 0});
        }
    }
    std::vector<tk::SvdItem> items;
    std::vector<int> roff{0};
    for (const auto& rd : rounds) {
      items.insert(items.end(), rd.begin(), rd.end());
      roff.push_back(static_cast<int>(items.size()));
    }
    DevBuf d_items, d_flags;
    d_items.upload(items);
    d_flags.alloc(std::max<size_t>(1, 2 * size_t(nsec)) * sizeof(int32_t));
    const tk::SvdSector* d_secs = static_cast<const tk::SvdSector*>(sv->secs.p);
    double* d_ws = static_cast<double*>(sv->ws.p);
    int32_t* flags = static_cast<int32_t*>(d_flags.p);
    hip_check(tk::launch_svd_init(d_secs, nsec, X, d_ws, st), "SVD init launch");
    // sweeps until a sweep rotates nothing (per sector: the sweeps used,
    // 0 while it still rotates)
    std::vector<int32_t> rotated(nsec), sweeps(nsec, 0);
    bool all_done = nsec == 0;
    for (int sw = 0; sw < kSvdMaxSweeps && !all_done; ++sw) {
      int32_t* cur = flags + (sw & 1) * nsec;
      const int32_t* prev = flags + ((sw + 1) & 1) * nsec;
      hip_check(hipMemsetAsync(cur, 0, nsec * sizeof(int32_t), st), "flag clear");
      for (size_t g = 0; g < rounds.size(); ++g)
        hip_check(tk::launch_svd_round(static_cast<const tk::SvdItem*>(d_items.p) + roff[g], roff[g + 1] - roff[g],
                                       d_secs, d_ws, prev, cur, sw, tol, st),
                  "SVD round launch");
      hip_check(hipMemcpyAsync(rotated.data(), cur, nsec * sizeof(int32_t), hipMemcpyDeviceToHost, st),
                "copy of the rotation flags");
      hip_check(hipStreamSynchronize(st), "stream synchronize");
      all_done = true;
      for (int r = 0; r < nsec; ++r) {
        if (sweeps[r] != 0) continue;
        if (rotated[r] == 0) sweeps[r] = sw + 1;
        else all_done = false;
      }
    }
    for (int r = 0; r < nsec; ++r) {
      sv->max_sweeps = std::max(sv->max_sweeps, sweeps[r] != 0 ? sweeps[r] : kSvdMaxSweeps);
      if (sweeps[r] == 0)
        fail(TK_ERR_UNSUPPORTED, "the Jacobi iteration of a " + std::to_string(sv->sec[r].m) + " x " +
                                     std::to_string(sv->sec[r].n) + " sector did not converge in " +
                                     std::to_string(kSvdMaxSweeps) + " sweeps");
    }
    hip_check(tk::launch_svd_finish(d_secs, nsec, d_ws, st), "SVD finish launch");
    hip_check(hipStreamSynchronize(st), "stream synchronize");
    int64_t nsig = 0;
    for (const auto& r : sv->sec) nsig += r.n;
    std::vector<double> sig(nsig);
    if (nsig)
      hip_check(hipMemcpy(sig.data(), d_ws + sv->sec.front().s, nsig * sizeof(double), hipMemcpyDeviceToHost),
                "copy of the singular values");
    sv->sigma = sig;
    // the largest values over all sectors (ties: sector order, then index)
    struct Val {
      double s;
      int32_t r, j;
    };
    std::vector<Val> all;
    int64_t base = 0;
    for (size_t r = 0; r < sv->sec.size(); ++r) {
      for (int j = 0; j < sv->sec[r].n; ++j) all.push_back({sv->sigma[base + j], static_cast<int32_t>(r), j});
      base += sv->sec[r].n;
    }
    std::stable_sort(all.begin(), all.end(), [](const Val& a, const Val& b) {
      return a.s != b.s ? a.s > b.s : (a.r != b.r ? a.r < b.r : a.j < b.j);
    });
    size_t nkeep = 0;
    while (nkeep < all.size() && all[nkeep].s > cutoff && (max_dim < 0 || int64_t(nkeep) < max_dim)) ++nkeep;
    double e2 = 0.0;
    for (size_t i = nkeep; i < all.size(); ++i) e2 += all[i].s * all[i].s;
    sv->err = std::sqrt(e2);
    sv->keep.assign(sv->sec.size(), {});
    for (size_t i = 0; i < nkeep; ++i) sv->keep[all[i].r].push_back(all[i].j);
    std::vector<int32_t> ks;
    std::vector<int64_t> kd;
    for (size_t r = 0; r < sv->sec.size(); ++r)
      if (!sv->keep[r].empty()) {
        ks.push_back(sv->sec_sector[r]);
        kd.push_back(static_cast<int64_t>(sv->keep[r].size()));
      }
    if (ks.empty()) fail(TK_ERR_INVALID_ARG, "the truncation keeps no singular value");
    const Space W = bond_space(T, ks, kd);
    sv->U = get_structure(T.sym, T.cod, {W});
    sv->S = get_structure(T.sym, {W}, {W});
    sv->V = get_structure(T.sym, {W}, T.dom);
    *out = sv.release();
  });
}

tk_status tk_svd_create_factor(tk_context* ctx, const tk_svd* svd, int32_t which, void* device_buf,
                               uint64_t buf_bytes, tk_tensor** out) {
  return guarded([&] {
    if (!svd || !out || which < 0 || which > 2) fail(TK_ERR_INVALID_ARG, "bad factor request");
    const auto& st = which == 0 ? svd->U : which == 1 ? svd->S : svd->V;
    *out = new_tensor(ctx, st, TK_F64, device_buf, buf_bytes);
  });
}

tk_status tk_svd_finish(tk_svd* svd, tk_tensor* U, tk_tensor* S, tk_tensor* Vh, double* trunc_err, void* stream) {
  return guarded([&] {
    if (!svd || !U || !S || !Vh) fail(TK_ERR_INVALID_ARG, "null argument");
    auto same = [](const tk_tensor* t, const std::shared_ptr<Structure>& st) {
      return t->st == st || t->st->sig == st->sig;
    };
    if (!same(U, svd->U) || !same(S, svd->S) || !same(Vh, svd->V))
      fail(TK_ERR_SPACE_MISMATCH, "factor tensors do not have the SVD's spaces");
    if (U->dtype != TK_F64 || S->dtype != TK_F64 || Vh->dtype != TK_F64) fail(TK_ERR_DTYPE, "factors are fp64");
    for (const tk_tensor* t : {U, S, Vh})
      if (!t->data && t->st->size) fail(TK_ERR_INVALID_ARG, "factor without data");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hip_check(hipMemsetAsync(S->data, 0, S->st->size * sizeof(double), st), "clear of S");
    // copies: U columns, rows of Vh, the diagonal of S (sources in the workspace, buffer 0)
    TaskList tl;
    const Structure &Us = *svd->U, &Ss = *svd->S, &Vs = *svd->V;
    for (size_t r = 0; r < svd->sec.size(); ++r) {
      const auto& kp = svd->keep[r];
      if (kp.empty()) continue;
      const tk::SvdSector& sc = svd->sec[r];
      const int64_t key = svd->T->keys[svd->sec_sector[r]];
      const int su = Us.sector_of_key(key), ss = Ss.sector_of_key(key), sv = Vs.sector_of_key(key);
      if (su < 0 || ss < 0 || sv < 0) fail(TK_ERR_SPACE_MISMATCH, "internal: factor lacks a sector");
      const int64_t k = static_cast<int64_t>(kp.size());
      for (int64_t i = 0; i < k; ++i) {
        const int j = kp[i];
        int64_t dim[1], one[1] = {1}, ds[1];
        // U(:, i) <- left vector j: a column of W, or of V for a transposed matrix
        dim[0] = sc.R;
        ds[0] = 1;
        add_block_tasks(tl, 0, sc.trans ? sc.v + int64_t(j) * sc.n : sc.w + int64_t(j) * sc.m, 1,
                        Us.soff[su] + i * sc.R, 1, dim, one, ds, 1.0f);
        // Vh(i, :) <- right vector j: a column of V, or of W for a transposed matrix
        dim[0] = sc.C;
        ds[0] = k;
        add_block_tasks(tl, 0, sc.trans ? sc.w + int64_t(j) * sc.m : sc.v + int64_t(j) * sc.n, 3,
                        Vs.soff[sv] + i, 1, dim, one, ds, 1.0f);
        dim[0] = 1;
        ds[0] = 1;
        add_block_tasks(tl, 0, sc.s + j, 2, Ss.soff[ss] + i * (k + 1), 1, dim, one, ds, 1.0f);
      }
    }
    pack_workgroups(tl);
    tl.upload();
    tk::Ptrs ptrs{};
    ptrs.p[0] = svd->ws.p;
    ptrs.p[1] = U->data;
    ptrs.p[2] = S->data;
    ptrs.p[3] = Vh->data;
    launch_tasklist(TK_F64, tl, ptrs, 1.0, 0.0, st, false, "factor copy launch");
    hip_check(hipStreamSynchronize(st), "stream synchronize");  // tl is freed on return
    if (trunc_err) *trunc_err = svd->err;
  });
}

tk_status tk_svd_info(const tk_svd* svd, int64_t* nsectors, int64_t* nkept, int32_t* max_sweeps) {
  return guarded([&] {
    if (!svd) fail(TK_ERR_INVALID_ARG, "null argument");
    int64_t k = 0;
    for (const auto& v : svd->keep) k += static_cast<int64_t>(v.size());
    if (nsectors) *nsectors = static_cast<int64_t>(svd->sec.size());
    if (nkept) *nkept = k;
    if (max_sweeps) *max_sweeps = svd->max_sweeps;
  });
}

tk_status tk_svd_destroy(tk_svd* svd) {
  return guarded([&] { delete svd; });
}

tk_status tk_tensor_trace(tk_context* ctx, const tk_tensor* A, const int32_t* p, int32_t np, const int32_t* q,
                          int32_t nq, const int32_t* t1, const int32_t* t2, int32_t nt, double alpha, double beta,
                          tk_tensor* C, void* stream) {
  return guarded([&] {
    if (!ctx || !A || !C) fail(TK_ERR_INVALID_ARG, "null argument");
    if (A->dtype != C->dtype) fail(TK_ERR_DTYPE, "dtype mismatch");
    if (!A->data && A->st->size) fail(TK_ERR_INVALID_ARG, "A has no data");
    if (!C->data && C->st->size) fail(TK_ERR_INVALID_ARG, "C has no data");
    if (A->data && A->data == C->data) fail(TK_ERR_INVALID_ARG, "C aliases A");
    auto pv = to_vec(p, np, "p"), qv = to_vec(q, nq, "q"), a = to_vec(t1, nt, "t1"), b = to_vec(t2, nt, "t2");
    check_trace_lists(*A->st, pv, qv, a, b);
    std::vector<Space> c, d;
    permute_spaces(*A->st, pv, qv, c, d);
    if (c != C->st->cod || d != C->st->dom) fail(TK_ERR_SPACE_MISMATCH, "C does not have the traced spaces");
    std::string key = "T#" + A->st->sig + "#" + C->st->sig + "#";
    for (const auto* v : {&pv, &qv, &a, &b}) {
      for (int x : *v) key += std::to_string(x) + ",";
      key += "/";
    }
    std::shared_ptr<TracePlan> tp;
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      auto it = ctx->trace_plans.find(key);
      if (it != ctx->trace_plans.end()) tp = it->second;
    }
    if (!tp) {
      tp = std::make_shared<TracePlan>();
      tp->A = A->st;
      tp->C = C->st;
      plan_trace_tasks(*A->st, pv, qv, a, b, *C->st, *tp);
      tp->tl.upload();
      tp->d_contribs.upload(tp->contribs);
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->trace_plans[key] = tp;
    }
    tk::Ptrs ptrs{};
    ptrs.p[tk::kBufA] = A->data;
    ptrs.p[tk::kBufC] = C->data;
    hip_check(tk::launch_trace(A->dtype, static_cast<const tk::TraceTask*>(tp->tl.d_tasks.p),
                               static_cast<const int32_t*>(tp->tl.d_wg.p), tp->tl.nwg(),
                               static_cast<const tk::TraceContrib*>(tp->d_contribs.p), ptrs, alpha, beta, false,
                               static_cast<hipStream_t>(stream)),
              "trace launch");
  });
}

tk_status tk_tensor_adjoint(tk_context* ctx, const tk_tensor* A, tk_tensor* C, void* stream) {
  return guarded([&] {
    if (!ctx || !A || !C) fail(TK_ERR_INVALID_ARG, "null argument");
    if (A->dtype != C->dtype) fail(TK_ERR_DTYPE, "dtype mismatch");
    if (C->st->cod != A->st->dom || C->st->dom != A->st->cod) fail(TK_ERR_SPACE_MISMATCH, "C is not shaped as A^dagger");
    if (A->data && A->data == C->data) fail(TK_ERR_INVALID_ARG, "C aliases A");
    const std::string key = "ADJ#" + A->st->sig;
    std::shared_ptr<PermPlan> pp;
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      auto it = ctx->perm_plans.find(key);
      if (it != ctx->perm_plans.end()) pp = it->second;
    }
    if (!pp) {
      pp = std::make_shared<PermPlan>();
      const Structure& sA = *A->st;
      const Structure& sC = *C->st;
      for (size_t s = 0; s < sA.keys.size(); ++s) {
        const int sc = sC.sector_of_key(sA.keys[s]);
        if (sc < 0) fail(TK_ERR_SPACE_MISMATCH, "internal: adjoint sector missing");
        // C^c = (A^c)^T: output (i', j') <- input (j', i')
        int64_t dims[2] = {sA.C[s], sA.R[s]}, ss[2] = {sA.R[s], 1}, ds[2] = {1, sC.R[sc]};
        add_block_tasks(pp->tl, tk::kBufA, sA.soff[s], tk::kBufC, sC.soff[sc], 2, dims, ss, ds, 1.0f);
      }
      pack_workgroups(pp->tl);
      pp->tl.upload();
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->perm_plans[key] = pp;
    }
    tk::Ptrs ptrs{};
    ptrs.p[tk::kBufA] = A->data;
    ptrs.p[tk::kBufC] = C->data;
    launch_tasklist(A->dtype, pp->tl, ptrs, 1.0, 0.0, static_cast<hipStream_t>(stream), false, "adjoint launch");
  });
}

tk_status tk_plan_contract(tk_context* ctx, const tk_tensor* A, const int32_t* pA, int32_t npA, const int32_t* qA,
                           int32_t nqA, const tk_tensor* B, const int32_t* pB, int32_t npB, const int32_t* qB,
                           int32_t nqB, const int32_t* pAB, int32_t npAB, const int32_t* qAB, int32_t nqAB,
                           int32_t precision, const tk_tensor* C, tk_plan** out) {
  return guarded([&] {
    if (!A || !B || !C || !out) fail(TK_ERR_INVALID_ARG, "null argument");
    auto P = build_contract_plan(ctx, A, to_vec(pA, npA, "pA"), to_vec(qA, nqA, "qA"), B, to_vec(pB, npB, "pB"),
                                 to_vec(qB, nqB, "qB"), to_vec(pAB, npAB, "pAB"), to_vec(qAB, nqAB, "qAB"), precision, C);
    *out = P.release();
  });
}

tk_status tk_plan_execute(tk_plan* plan, const tk_tensor* A, const tk_tensor* B, tk_tensor* C, double alpha,
                          double beta, void* stream) {
  return guarded([&] {
    if (!plan) fail(TK_ERR_INVALID_ARG, "null plan");
    execute_plan(*plan, A, B, C, alpha, beta, static_cast<hipStream_t>(stream));
  });
}

tk_status tk_plan_execute_stages(tk_plan* plan, const tk_tensor* A, const tk_tensor* B, tk_tensor* C, double alpha,
                                 double beta, int32_t stages, void* stream) {
  return guarded([&] {
    if (!plan) fail(TK_ERR_INVALID_ARG, "null plan");
    if (stages < 0 || stages > (TK_STAGE_ALL | TK_STAGE_PERMUTE_A | TK_STAGE_PERMUTE_B))
      fail(TK_ERR_INVALID_ARG, "bad stage mask");
    execute_plan(*plan, A, B, C, alpha, beta, static_cast<hipStream_t>(stream), stages);
  });
}

tk_status tk_plan_destroy(tk_plan* plan) {
  return guarded([&] { delete plan; });
}

tk_status tk_plan_info(const tk_plan* plan, int64_t* ngemm, double* flops, int64_t* nzero, int64_t* workspace_bytes,
                       int32_t* tile_m, int32_t* tile_n, int32_t* tile_k) {
  return guarded([&] {
    if (!plan) fail(TK_ERR_INVALID_ARG, "null plan");
    if (ngemm) *ngemm = static_cast<int64_t>(plan->mnk.size() / 3);
    if (flops) *flops = plan->flops;
    if (nzero) *nzero = plan->nzero;
    if (workspace_bytes) {
      const int64_t es = plan->dtype == TK_F64 ? 8 : 4;
      *workspace_bytes = (plan->needA ? plan->At->size * es : 0) + (plan->needB ? plan->Bt->size * es : 0) +
                         (plan->post ? plan->Ct->size * es : 0) + 4 * (plan->planeA + plan->planeB);
    }
    if (tile_m) *tile_m = plan->tile_m;
    if (tile_n) *tile_n = plan->tile_n;
    if (tile_k) *tile_k = plan->tile_k;
  });
}

tk_status tk_plan_counts(const tk_plan* plan, int64_t* c) {
  return guarded([&] {
    if (!plan || !c) fail(TK_ERR_INVALID_ARG, "null argument");
    const tk_plan& P = *plan;
    int64_t skt = 0, skw = 0;
    for (const auto& l : P.smallk) {
      skt += static_cast<int64_t>(l.tasks.size());
      skw += l.n();
    }
    for (const auto& l : P.skblocks) {
      skt += static_cast<int64_t>(l.tasks.size());
      skw += l.nwg();
    }
    int64_t nrun = 0, nrw = 0;
    for (const auto& r : P.skruns) {
      nrun += static_cast<int64_t>(r.runs.size());
      nrw += r.nwg();
    }
    const int64_t v[14] = {static_cast<int64_t>(P.pre.tasks.size() + P.pre.tiles.size()),
                           P.pre.nwg() + P.pre.ntiles(),
                           static_cast<int64_t>(P.zero.tasks.size() + P.zranges.ranges.size()),
                           P.zero.nwg() + P.zranges.nwg(), skt, skw,
                           static_cast<int64_t>(P.descs.size()), static_cast<int64_t>(P.tiles.size()),
                           static_cast<int64_t>(P.wg_first.size()) - 1, P.ngroups, P.nslots,
                           static_cast<int64_t>(P.makespan + 0.5), nrun, nrw};
    std::copy(v, v + 14, c);
  });
}

tk_status tk_plan_gemms(const tk_plan* plan, int64_t first, int64_t count, int64_t* mnk) {
  return guarded([&] {
    if (!plan || !mnk) fail(TK_ERR_INVALID_ARG, "null argument");
    if (first < 0 || count < 0 || first + count > static_cast<int64_t>(plan->mnk.size() / 3))
      fail(TK_ERR_INVALID_ARG, "range out of bounds");
    std::copy(plan->mnk.begin() + 3 * first, plan->mnk.begin() + 3 * (first + count), mnk);
  });
}

tk_status tk_plan_worklist(const tk_plan* plan, int32_t kind, int64_t* counts, int64_t* vstart, int64_t* len,
                           int32_t* lin0, int32_t* shape, int32_t* first, int64_t* wstart, int32_t* dimrec) {
  return guarded([&] {
    if (!plan || !counts) fail(TK_ERR_INVALID_ARG, "null argument");
    if (kind < 0 || kind > 8) fail(TK_ERR_INVALID_ARG, "kind must be 0 (zero ranges) or a K value 1..8");
    const std::vector<int32_t>* fi;
    const std::vector<int64_t>* ws;
    int64_t total, n, nrec = 0;
    if (kind == 0) {
      const ZeroSet& z = plan->zranges;
      fi = &z.first;
      ws = &z.wstart;
      total = z.total;
      n = static_cast<int64_t>(z.ranges.size());
      for (int64_t i = 0; i < n; ++i) {
        if (vstart) vstart[i] = z.ranges[i].vstart;
        if (len) len[i] = (i + 1 < n ? z.ranges[i + 1].vstart : total) - z.ranges[i].vstart;
      }
    } else {
      const RunSet& r = plan->skruns[kind];
      fi = &r.first;
      ws = &r.wstart;
      total = r.total;
      n = static_cast<int64_t>(r.runs.size());
      nrec = static_cast<int64_t>(r.shapes.size());
      for (int64_t i = 0; i < n; ++i) {
        if (vstart) vstart[i] = r.runs[i].vstart;
        if (len) len[i] = r.runs[i].len;
        if (lin0) lin0[i] = r.runs[i].lin0;
        if (shape) shape[i] = r.runs[i].shape;
      }
      if (dimrec)
        for (int64_t i = 0; i < nrec; ++i) {
          const tk::SkRunShape& sh = r.shapes[i];
          int32_t* o = dimrec + 25 * i;
          o[0] = sh.nd;
          for (int d = 0; d < 8; ++d) {
            const bool used = d < sh.nd;
            o[1 + 3 * d] = used ? static_cast<int32_t>(sh.dim[d].dimshr & 0xffffff) : 0;
            o[2 + 3 * d] = used ? static_cast<int32_t>(sh.dim[d].mag) : 0;
            o[3 + 3 * d] = used ? static_cast<int32_t>(32 + (sh.dim[d].dimshr >> 24)) : 0;
          }
        }
    }
    const int64_t nwg = fi->empty() ? 0 : static_cast<int64_t>(fi->size()) - 1;
    if (first) std::copy(fi->begin(), fi->end(), first);
    if (wstart) std::copy(ws->begin(), ws->end(), wstart);
    counts[0] = n;
    counts[1] = nwg;
    counts[2] = nrec;
  });
}

tk_status tk_permute_map(const tk_tensor* A, const int32_t* p, int32_t np, const int32_t* q, int32_t nq,
                         const tk_tensor* C, int64_t* dst_block, int32_t* sign) {
  return guarded([&] {
    if (!A || !C || !dst_block || !sign) fail(TK_ERR_INVALID_ARG, "null argument");
    auto pv = to_vec(p, np, "p");
    auto qv = to_vec(q, nq, "q");
    check_perm(pv, qv, A->st->N());
    std::vector<Space> c, d;
    permute_spaces(*A->st, pv, qv, c, d);
    if (c != C->st->cod || d != C->st->dom) fail(TK_ERR_SPACE_MISMATCH, "C does not have the permuted spaces");
    TaskList dummy;
    std::vector<int64_t> m;
    std::vector<int32_t> sg;
    plan_permute_tasks(*A->st, pv, qv, *C->st, 0, 0, false, dummy, &m, &sg);
    std::copy(m.begin(), m.end(), dst_block);
    std::copy(sg.begin(), sg.end(), sign);
  });
}

tk_status tk_tensor_contract_noalloc(tk_context* ctx, const tk_tensor* A, const int32_t* pA, int32_t npA,
                                     const int32_t* qA, int32_t nqA, const tk_tensor* B, const int32_t* pB,
                                     int32_t npB, const int32_t* qB, int32_t nqB, const int32_t* pAB, int32_t npAB,
                                     const int32_t* qAB, int32_t nqAB, double alpha, double beta, int32_t precision,
                                     tk_tensor* C, void* stream) {
  return guarded([&] {
    if (!ctx || !A || !B || !C) fail(TK_ERR_INVALID_ARG, "null argument");
    auto pa = to_vec(pA, npA, "pA"), qa = to_vec(qA, nqA, "qA"), pb = to_vec(pB, npB, "pB"), qb = to_vec(qB, nqB, "qB");
    auto pab = to_vec(pAB, npAB, "pAB"), qab = to_vec(qAB, nqAB, "qAB");
    Scratch& S = scratch_of(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> g(S.mu);
    // the staging copy of the previous call must have left host memory
    // before the staging buffer is refilled
    if (S.pending) hip_check(hipEventSynchronize(S.copied), "hipEventSynchronize");
    S.pending = false;
    S.staging.clear();
    Arena arena;
    arena.staging = &S.staging;
    std::unique_ptr<tk_plan> P;
    {
      struct Active {
        explicit Active(Arena* a) { t_arena = a; }
        ~Active() { t_arena = nullptr; }
      } active(&arena);
      P = build_contract_plan(ctx, A, pa, qa, B, pb, qb, pab, qab, precision, C);
    }
    arena.place(static_cast<char*>(S.base), tk::kScratchBytes, st);
    hip_check(hipEventRecord(S.copied, st), "hipEventRecord");
    S.pending = true;
    execute_plan(*P, A, B, C, alpha, beta, st);
  });
}

uint64_t tk_device_alloc_count(void) { return g_device_allocs.load(std::memory_order_relaxed); }

tk_status tk_tensor_contract(tk_context* ctx, const tk_tensor* A, const int32_t* pA, int32_t npA, const int32_t* qA,
                             int32_t nqA, const tk_tensor* B, const int32_t* pB, int32_t npB, const int32_t* qB,
                             int32_t nqB, const int32_t* pAB, int32_t npAB, const int32_t* qAB, int32_t nqAB,
                             double alpha, double beta, int32_t precision, tk_tensor* C, void* stream) {
  return guarded([&] {
    if (!ctx || !A || !B || !C) fail(TK_ERR_INVALID_ARG, "null argument");
    auto pa = to_vec(pA, npA, "pA"), qa = to_vec(qA, nqA, "qA"), pb = to_vec(pB, npB, "pB"), qb = to_vec(qB, nqB, "qB");
    auto pab = to_vec(pAB, npAB, "pAB"), qab = to_vec(qAB, nqAB, "qAB");
    const std::string key = plan_key(A, pa, qa, B, pb, qb, pab, qab, precision, C);
    std::shared_ptr<tk_plan> P;
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      auto it = ctx->plans.find(key);
      if (it != ctx->plans.end()) P = it->second;
    }
    if (!P) {
      P = std::shared_ptr<tk_plan>(build_contract_plan(ctx, A, pa, qa, B, pb, qb, pab, qab, precision, C).release());
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->plans[key] = P;
    }
    execute_plan(*P, A, B, C, alpha, beta, static_cast<hipStream_t>(stream));
  });
}

tk_status tk_tile_shapes(int32_t* count, int32_t* tile_mnk) {
  return guarded([&] {
    if (!count) fail(TK_ERR_INVALID_ARG, "null count");
    *count = tk::num_tile_shapes();
    if (tile_mnk)
      for (int i = 0; i < *count; ++i) tk::tile_shape(i, &tile_mnk[3 * i], &tile_mnk[3 * i + 1], &tile_mnk[3 * i + 2]);
  });
}

tk_status tk_plan_set_tile(tk_plan* plan, int32_t tile_m, int32_t tile_n, int32_t tile_k) {
  return guarded([&] {
    if (!plan) fail(TK_ERR_INVALID_ARG, "null plan");
    if (!tk::gemm_tile_supported(plan->dtype, plan->precision, tile_m, tile_n, tile_k))
      fail(TK_ERR_UNSUPPORTED, "tile shape not available");
    plan_reschedule(*plan, tile_m, tile_n, tile_k);
  });
}

}  // extern "C"

namespace {

// Append the task list `src` of member plan i to `dst`, shifting buffer ids.
void merge_tasks(TaskList& dst, const TaskList& src, int member) {
  const int base = static_cast<int>(dst.tasks.size());
  for (PermTask t : src.tasks) {
    if (t.src_buf >= 0) t.src_buf = static_cast<int16_t>(t.src_buf + member * tk::kBufsPerPlan);
    t.dst_buf = static_cast<int16_t>(t.dst_buf + member * tk::kBufsPerPlan);
    dst.tasks.push_back(t);
  }
  for (size_t w = 1; w < src.wg_first.size(); ++w) dst.wg_first.push_back(base + src.wg_first[w]);
  for (tk::TileTask t : src.tiles) {
    if (t.src_buf >= 0) t.src_buf = static_cast<int16_t>(t.src_buf + member * tk::kBufsPerPlan);
    t.dst_buf = static_cast<int16_t>(t.dst_buf + member * tk::kBufsPerPlan);
    dst.tiles.push_back(t);
  }
}

void merge_smallk(SmallKSet& dst, const SmallKSet& src, int member, int32_t chan_base, int32_t pair_base) {
  for (tk::SmallKTask t : src.tasks) {
    t.a_buf = static_cast<int16_t>(t.a_buf + member * tk::kBufsPerPlan);
    t.b_buf = static_cast<int16_t>(t.b_buf + member * tk::kBufsPerPlan);
    t.dst_buf = static_cast<int16_t>(t.dst_buf + member * tk::kBufsPerPlan);
    t.rchan += chan_base;
    t.cchan += chan_base;
    t.pair += pair_base;
    dst.tasks.push_back(t);
  }
}

void batch_schedule(tk_batch& b, int tm, int tn, int tk) {
  b.tile_m = tm;
  b.tile_n = tn;
  b.tile_k = tk;
  Sched sc = schedule_tiles(b.descs, tm, tn, tk, b.ctx->num_cu, tk::gemm_blocks_per_cu(b.dtype, b.precision, tm, tn, tk),
                            b.precision);
  b.tiles = sc.tiles;
  b.wg_first = sc.wg_first;
  b.groups = sc.groups;
  b.ngroups = sc.ngroups;
  b.nslots = sc.nslots;
  upload_schedule(b.d_tiles, b.d_wg, b.d_partials, b.d_groups, sc, tm, tn);
}

void batch_launch_all(tk_batch& b, hipStream_t stream) {
  tk::Ptrs ptrs{};
  ptrs.table = static_cast<const uint64_t*>(b.d_table.p);
  launch_tasklist(b.dtype, b.pre, ptrs, 1.0, 0.0, stream, b.precision == TK_PREC_BF16X3, "permute launch");
  if (!b.descs.empty()) {
    tk::GemmArgs ga{};
    ga.descs = static_cast<const GemmDesc*>(b.d_descs.p);
    ga.tiles = static_cast<const GemmTile*>(b.d_tiles.p);
    ga.wg_first = static_cast<const int32_t*>(b.d_wg.p);
    ga.row_map = static_cast<const LegMap*>(b.d_rowmap.p);
    ga.col_map = static_cast<const LegMap*>(b.d_colmap.p);
    ga.pairs = static_cast<const PairDesc*>(b.d_pairs.p);
    ga.partials = static_cast<double*>(b.d_partials.p);
    ga.ptrs = ptrs;
    ga.alpha = b.alpha;
    ga.beta = b.beta;
    hip_check(tk::launch_gemm(b.dtype, b.precision, b.tile_m, b.tile_n, b.tile_k, ga,
                              static_cast<int>(b.wg_first.size()) - 1, stream),
              "gemm launch");
    hip_check(tk::launch_splitk_reduce(b.dtype, b.precision, b.tile_m, b.tile_n, b.tile_k, ga,
                                       static_cast<const GemmTile*>(b.d_groups.p), b.ngroups, stream),
              "split-K reduce launch");
  }
  for (int K = 1; K <= kSmallK; ++K)
    if (b.smallk[K].n() > 0)
      hip_check(tk::launch_smallk(b.dtype, b.precision, K, static_cast<const tk::SmallKTask*>(b.smallk[K].d_tasks.p),
                                  b.smallk[K].n(), static_cast<const tk::SkChan*>(b.d_skchans.p),
                                  static_cast<const PairDesc*>(b.d_skpairs.p), ptrs, b.alpha, b.beta, stream),
                "small-K launch");
  for (int K = 1; K <= kSmallK; ++K)
    if (b.skblocks[K].nwg() > 0)
      hip_check(tk::launch_smallk_blocks(b.dtype, b.precision, K,
                                         static_cast<const tk::SkBlockTask*>(b.skblocks[K].d_tasks.p),
                                         static_cast<const int32_t*>(b.skblocks[K].d_wg.p), b.skblocks[K].nwg(),
                                         static_cast<const tk::SkChan*>(b.d_skchans.p),
                                         static_cast<const PairDesc*>(b.d_skpairs.p), ptrs, b.alpha, b.beta, stream),
                "small-K block launch");
  for (int K = 1; K <= kSmallK; ++K)
    if (b.skruns[K].nwg() > 0)
      hip_check(tk::launch_smallk_runs(b.dtype, b.precision, K, static_cast<const tk::SkRun*>(b.skruns[K].d_runs.p),
                                       static_cast<int>(b.skruns[K].runs.size()),
                                       static_cast<const int32_t*>(b.skruns[K].d_first.p),
                                       static_cast<const int64_t*>(b.skruns[K].d_wstart.p), b.skruns[K].nwg(),
                                       static_cast<const tk::SkRunShape*>(b.skruns[K].d_shapes.p), ptrs, b.alpha, b.beta,
                                       stream),
                "small-K run launch");
  if (b.zranges.nwg() > 0)
    hip_check(tk::launch_zero_ranges(b.dtype, static_cast<const tk::ZeroRange*>(b.zranges.d_ranges.p),
                                     static_cast<int>(b.zranges.ranges.size()),
                                     static_cast<const int32_t*>(b.zranges.d_first.p),
                                     static_cast<const int64_t*>(b.zranges.d_wstart.p), b.zranges.nwg(), ptrs, b.beta, stream),
              "zero-range launch");
  launch_tasklist(b.dtype, b.zero, ptrs, b.alpha, b.beta, stream, false, "zero launch");
}

}  // namespace

extern "C" {

tk_status tk_batch_create(tk_context* ctx, tk_plan* const* plans, const tk_tensor* const* A, const tk_tensor* const* B,
                          tk_tensor* const* C, int32_t n, double alpha, double beta, tk_batch** out) {
  return guarded([&] {
    if (!ctx || !plans || !A || !B || !C || !out || n < 1) fail(TK_ERR_INVALID_ARG, "bad batch arguments");
    auto b = std::make_unique<tk_batch>();
    b->ctx = ctx;
    b->n = n;
    b->alpha = alpha;
    b->beta = beta;
    b->dtype = plans[0]->dtype;
    b->precision = plans[0]->precision;
    std::vector<uint64_t> table;
    for (int i = 0; i < n; ++i) {
      tk_plan& P = *plans[i];
      if (!P.ctx) fail(TK_ERR_INVALID_ARG, "batch member plan made without a context");
      if (P.dtype != b->dtype || P.precision != b->precision) fail(TK_ERR_DTYPE, "batch members differ in dtype / precision");
      if (P.post) fail(TK_ERR_UNSUPPORTED, "batch members need a fusable output permute (<= 4 legs per side)");
      check_exec_tensor(A[i], P.A, P.dtype, "A");
      check_exec_tensor(B[i], P.B, P.dtype, "B");
      check_exec_tensor(C[i], P.C, P.dtype, "C");
      const size_t es = A[i]->esize();
      auto wa = std::make_unique<DevBuf>(), wb = std::make_unique<DevBuf>();
      auto wap = std::make_unique<DevBuf>(), wbp = std::make_unique<DevBuf>();
      if (P.needA) wa->alloc(P.At->size * es);
      if (P.needB) wb->alloc(P.Bt->size * es);
      if (P.planeA) wap->alloc(4 * P.planeA);
      if (P.planeB) wbp->alloc(4 * P.planeB);
      // one entry per buffer id (kBufA .. kBufBp)
      table.push_back(reinterpret_cast<uint64_t>(A[i]->data));
      table.push_back(reinterpret_cast<uint64_t>(B[i]->data));
      table.push_back(reinterpret_cast<uint64_t>(C[i]->data));
      table.push_back(reinterpret_cast<uint64_t>(wa->p));
      table.push_back(reinterpret_cast<uint64_t>(wb->p));
      table.push_back(0);
      table.push_back(reinterpret_cast<uint64_t>(wap->p));
      table.push_back(reinterpret_cast<uint64_t>(wbp->p));
      static_assert(tk::kBufsPerPlan == 8, "batch table layout");
      b->ws.push_back(std::move(wa));
      b->ws.push_back(std::move(wb));
      b->ws.push_back(std::move(wap));
      b->ws.push_back(std::move(wbp));
      merge_tasks(b->pre, P.pre, i);
      merge_tasks(b->zero, P.zero, i);
      for (const auto& r : P.zranges.raw)
        b->zranges.add(std::get<0>(r) + i * tk::kBufsPerPlan, std::get<1>(r), std::get<2>(r));
      const int32_t skc = static_cast<int32_t>(b->skchans.size()), skp = static_cast<int32_t>(b->skpairs.size());
      for (int K = 1; K <= kSmallK; ++K) {
        merge_smallk(b->smallk[K], P.smallk[K], i, skc, skp);
        const int base = static_cast<int>(b->skblocks[K].tasks.size());
        for (tk::SkBlockTask t : P.skblocks[K].tasks) {
          t.a_buf = static_cast<int16_t>(t.a_buf + i * tk::kBufsPerPlan);
          t.b_buf = static_cast<int16_t>(t.b_buf + i * tk::kBufsPerPlan);
          t.dst_buf = static_cast<int16_t>(t.dst_buf + i * tk::kBufsPerPlan);
          t.rchan += skc;
          t.cchan += skc;
          t.pair += skp;
          b->skblocks[K].tasks.push_back(t);
        }
        for (size_t w = 1; w < P.skblocks[K].wg_first.size(); ++w)
          b->skblocks[K].wg_first.push_back(base + P.skblocks[K].wg_first[w]);
        const int32_t db = static_cast<int32_t>(b->skruns[K].shapes.size());
        b->skruns[K].shapes.insert(b->skruns[K].shapes.end(), P.skruns[K].shapes.begin(), P.skruns[K].shapes.end());
        for (tk::SkRun r : P.skruns[K].runs) {
          r.shape += db;
          r.buf = static_cast<int16_t>(r.buf + i * tk::kBufsPerPlan);
          r.a_buf = static_cast<int16_t>(r.a_buf + i * tk::kBufsPerPlan);
          r.b_buf = static_cast<int16_t>(r.b_buf + i * tk::kBufsPerPlan);
          b->skruns[K].runs.push_back(r);
        }
      }
      b->skchans.insert(b->skchans.end(), P.skchans.begin(), P.skchans.end());
      b->skpairs.insert(b->skpairs.end(), P.skpairs.begin(), P.skpairs.end());
      const int32_t rb = static_cast<int32_t>(b->row_map.size()), cb = static_cast<int32_t>(b->col_map.size());
      const int32_t pb = static_cast<int32_t>(b->pairs.size());
      for (GemmDesc d : P.descs) {
        d.a_buf = static_cast<int16_t>(d.a_buf + i * tk::kBufsPerPlan);
        d.b_buf = static_cast<int16_t>(d.b_buf + i * tk::kBufsPerPlan);
        d.c_buf = static_cast<int16_t>(d.c_buf + i * tk::kBufsPerPlan);
        if (d.mode == 1) {
          d.row_map += rb;
          d.col_map += cb;
          d.pair_base += pb;
        }
        b->descs.push_back(d);
      }
      b->row_map.insert(b->row_map.end(), P.row_map.begin(), P.row_map.end());
      b->col_map.insert(b->col_map.end(), P.col_map.begin(), P.col_map.end());
      b->pairs.insert(b->pairs.end(), P.pairs.begin(), P.pairs.end());
      b->flops += P.flops;
    }
    if (b->descs.size() > static_cast<size_t>(INT32_MAX)) fail(TK_ERR_UNSUPPORTED, "too many GEMMs");
    int tm, tn, tkk;
    choose_default_tile(b->descs, b->precision, &tm, &tn, &tkk);
    batch_schedule(*b, tm, tn, tkk);
    b->zranges.finalize();
    for (auto& r : b->skruns) r.finalize();
    b->pre.upload();
    b->zero.upload();
    b->zranges.upload();
    for (auto& l : b->smallk) l.upload();
    for (auto& l : b->skblocks) l.upload();
    for (auto& r : b->skruns) r.upload();
    b->d_skchans.upload(b->skchans);
    b->d_skpairs.upload(b->skpairs);
    b->d_descs.upload(b->descs);
    b->d_rowmap.upload(b->row_map);
    b->d_colmap.upload(b->col_map);
    b->d_pairs.upload(b->pairs);
    b->d_table.upload(table);
    *out = b.release();
  });
}

tk_status tk_batch_launch(tk_batch* batch, void* stream) {
  return guarded([&] {
    if (!batch) fail(TK_ERR_INVALID_ARG, "null batch");
    batch_launch_all(*batch, static_cast<hipStream_t>(stream));
  });
}

tk_status tk_batch_capture(tk_batch* batch, void* stream) {
  return guarded([&] {
    if (!batch) fail(TK_ERR_INVALID_ARG, "null batch");
    if (!stream) fail(TK_ERR_INVALID_ARG, "graph capture needs a non-null stream");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (batch->exec) {
      (void)hipGraphExecDestroy(batch->exec);
      batch->exec = nullptr;
    }
    if (batch->graph) {
      (void)hipGraphDestroy(batch->graph);
      batch->graph = nullptr;
    }
    hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      batch_launch_all(*batch, s);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hip_check(hipStreamEndCapture(s, &batch->graph), "hipStreamEndCapture");
    hip_check(hipGraphInstantiate(&batch->exec, batch->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  });
}

tk_status tk_batch_replay(tk_batch* batch, void* stream) {
  return guarded([&] {
    if (!batch || !batch->exec) fail(TK_ERR_INVALID_ARG, "batch has no captured graph");
    hip_check(hipGraphLaunch(batch->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
  });
}

tk_status tk_batch_info(const tk_batch* batch, int64_t* ngemm, int64_t* ntiles, double* flops, int32_t* tile_m,
                        int32_t* tile_n, int32_t* tile_k) {
  return guarded([&] {
    if (!batch) fail(TK_ERR_INVALID_ARG, "null batch");
    if (ngemm) *ngemm = static_cast<int64_t>(batch->descs.size());
    if (ntiles) *ntiles = static_cast<int64_t>(batch->tiles.size());
    if (flops) *flops = batch->flops;
    if (tile_m) *tile_m = batch->tile_m;
    if (tile_n) *tile_n = batch->tile_n;
    if (tile_k) *tile_k = batch->tile_k;
  });
}

tk_status tk_batch_set_tile(tk_batch* batch, int32_t tile_m, int32_t tile_n, int32_t tile_k) {
  return guarded([&] {
    if (!batch) fail(TK_ERR_INVALID_ARG, "null batch");
    if (!tk::gemm_tile_supported(batch->dtype, batch->precision, tile_m, tile_n, tile_k))
      fail(TK_ERR_UNSUPPORTED, "tile shape not available");
    batch_schedule(*batch, tile_m, tile_n, tile_k);
    if (batch->exec) {
      (void)hipGraphExecDestroy(batch->exec);
      batch->exec = nullptr;
    }
    if (batch->graph) {
      (void)hipGraphDestroy(batch->graph);
      batch->graph = nullptr;
    }
  });
}

tk_status tk_batch_destroy(tk_batch* batch) {
  return guarded([&] { delete batch; });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// SU(2) leg permutation
// ---------------------------------------------------------------------------
struct tk_su2_plan {
  su2::Plan P;
};

tk_status tk_su2_plan_create_dual(int32_t n1, int32_t n2, const int32_t* nsec, const int32_t* twoj,
                                  const int64_t* deg, const int32_t* isdual, const int32_t* p, int32_t np,
                                  const int32_t* q, int32_t nq, tk_su2_plan** out) {
  return guarded([&] {
    if (!out || !nsec || !twoj || !deg || !p || !q) fail(TK_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (n1 < 1 || n2 < 1) fail(TK_ERR_INVALID_ARG, "codomain and domain need at least one leg each");
    if (n1 + n2 > tk::kMaxDims) fail(TK_ERR_UNSUPPORTED, "more than 8 legs");
    if (np < 1 || nq < 1 || np + nq != n1 + n2) fail(TK_ERR_INVALID_ARG, "p and q must split the legs, both non-empty");
    auto plan = std::make_unique<tk_su2_plan>();
    std::vector<su2::Leg> legs;
    int64_t k = 0;
    for (int l = 0; l < n1 + n2; ++l) {
      if (nsec[l] < 1 || nsec[l] > 64) fail(TK_ERR_INVALID_ARG, "a leg needs 1..64 sectors");
      su2::Leg leg;
      leg.dual = isdual && isdual[l] != 0;
      for (int i = 0; i < nsec[l]; ++i, ++k) {
        if (twoj[k] < 0 || twoj[k] > 64) fail(TK_ERR_CHARGE, "spin (twice its value) outside 0..64");
        if (i > 0 && twoj[k] <= leg.tj.back()) fail(TK_ERR_CHARGE, "spins of a leg must be strictly ascending");
        if (deg[k] < 1 || deg[k] > INT32_MAX) fail(TK_ERR_INVALID_ARG, "degeneracy outside 1..2^31-1");
        leg.tj.push_back(twoj[k]);
        leg.deg.push_back(deg[k]);
      }
      legs.push_back(leg);
      (l < n1 ? plan->P.A.cod : plan->P.A.dom).push_back(std::move(leg));
    }
    std::vector<int> order(p, p + np), seen(n1 + n2, 0);
    order.insert(order.end(), q, q + nq);
    for (int x : order)
      if (x < 0 || x >= n1 + n2 || seen[x]++) fail(TK_ERR_INVALID_ARG, "(p, q) must list every leg once");
    bool crossing = false;
    for (int m = 0; m < n1 + n2; ++m) {
      su2::Leg leg = legs[order[m]];
      const bool crossed = (order[m] < n1) != (m < np);
      crossing = crossing || crossed;
      leg.dual = leg.dual != crossed;  // a leg changing sides turns into the dual space
      (m < np ? plan->P.C.cod : plan->P.C.dom).push_back(std::move(leg));
    }
    plan->P.A.build();
    plan->P.C.build();
    bool anydual = false;
    for (const auto& l : legs) anydual = anydual || l.dual;
    if (crossing || anydual) {
      su2::plan_transpose(plan->P, order);
    } else {
      std::vector<int> pv(p, p + np), qv(q, q + nq);
      su2::plan_permute(plan->P, pv, qv);
    }
    // device tables go to the current device now, so launches allocate
    // nothing (and may be captured); without a device the plan is host only
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
      int dev = 0;
      hip_check(hipGetDevice(&dev), "hipGetDevice");
      plan->P.tl.upload();
      plan->P.d_contribs.upload(plan->P.contribs);
      plan->P.device = dev;
    } else {
      (void)hipGetLastError();
    }
    *out = plan.release();
  });
}

tk_status tk_su2_plan_create(int32_t n1, int32_t n2, const int32_t* nsec, const int32_t* twoj, const int64_t* deg,
                             const int32_t* p, const int32_t* q, tk_su2_plan** out) {
  return tk_su2_plan_create_dual(n1, n2, nsec, twoj, deg, nullptr, p, n1, q, n2, out);
}

tk_status tk_su2_plan_legs(const tk_su2_plan* plan, int32_t* n1, int32_t* n2, int32_t* isdual) {
  return guarded([&] {
    if (!plan) fail(TK_ERR_INVALID_ARG, "null plan");
    const auto& C = plan->P.C;
    if (n1) *n1 = static_cast<int32_t>(C.cod.size());
    if (n2) *n2 = static_cast<int32_t>(C.dom.size());
    if (isdual) {
      int k = 0;
      for (const auto& l : C.cod) isdual[k++] = l.dual;
      for (const auto& l : C.dom) isdual[k++] = l.dual;
    }
  });
}

tk_status tk_su2_plan_info(const tk_su2_plan* plan, int64_t* in_size, int64_t* out_size, int64_t* ncontrib) {
  return guarded([&] {
    if (!plan) fail(TK_ERR_INVALID_ARG, "null plan");
    if (in_size) *in_size = plan->P.A.size;
    if (out_size) *out_size = plan->P.C.size;
    if (ncontrib) *ncontrib = static_cast<int64_t>(plan->P.contribs.size());
  });
}

tk_status tk_su2_plan_contribs(const tk_su2_plan* plan, int64_t cap, int64_t* dst, int64_t* src, double* coef) {
  return guarded([&] {
    if (!plan || !dst || !src || !coef) fail(TK_ERR_INVALID_ARG, "null argument");
    const auto& P = plan->P;
    if (cap < static_cast<int64_t>(P.contribs.size())) fail(TK_ERR_INVALID_ARG, "cap below the contribution count");
    for (size_t i = 0; i < P.contribs.size(); ++i) {
      dst[i] = P.tab_dst[i];
      src[i] = P.tab_src[i];
      coef[i] = P.contribs[i].coef;
    }
  });
}

tk_status tk_su2_permute(tk_su2_plan* plan, int32_t dtype, const void* A, void* C, double alpha, double beta,
                         void* stream) {
  return guarded([&] {
    if (!plan) fail(TK_ERR_INVALID_ARG, "null plan");
    if (dtype != TK_F64 && dtype != TK_F32) fail(TK_ERR_DTYPE, "dtype must be TK_F64 or TK_F32");
    auto& P = plan->P;
    if (!A && P.A.size) fail(TK_ERR_INVALID_ARG, "A is null");
    if (!C && P.C.size) fail(TK_ERR_INVALID_ARG, "C is null");
    if (A && A == C) fail(TK_ERR_INVALID_ARG, "C aliases A");
    if (P.device < 0) fail(TK_ERR_INVALID_ARG, "the plan was created without a HIP device (host only)");
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (P.device != dev) fail(TK_ERR_INVALID_ARG, "the plan's tables live on another device");
    tk::Ptrs ptrs{};
    ptrs.p[tk::kBufA] = const_cast<void*>(A);
    ptrs.p[tk::kBufC] = C;
    hip_check(tk::launch_trace(dtype, static_cast<const tk::TraceTask*>(P.tl.d_tasks.p),
                               static_cast<const int32_t*>(P.tl.d_wg.p), P.tl.nwg(),
                               static_cast<const tk::TraceContrib*>(P.d_contribs.p), ptrs, alpha, beta, P.gather,
                               static_cast<hipStream_t>(stream)),
              "SU(2) permute launch");
  });
}

tk_status tk_su2_plan_destroy(tk_su2_plan* plan) {
  return guarded([&] { delete plan; });
}

// Host planner of the tnrcs library: builds the circuit's tensor network,
// folds small slice-local subtrees in FP64, and turns the caller's pairwise
// order into a per-slice kernel sequence with tensor layouts and arena
// offsets.
//
// Paper anchors: the network of an amplitude (main text, customized-TNC
// section; Supplement Fig. S2); pre-absorbing low-rank tensors (Supplement,
// TNC section); index slicing as a sum of smaller networks (main text); each
// pairwise contraction as permutation + matrix product (Supplement
// Eq. (matmul)) or the fused skewed form (Supplement Fig. S7a).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <iomanip>
#include <sstream>

#include "internal.h"

namespace tnrcs {

using cd = std::complex<double>;

bool make_runs(const std::vector<int>& pos, Runs* r) {
  r->n = 0;
  int j = 0;
  const int n = (int)pos.size();
  while (j < n) {
    int len = 1;
    while (j + len < n && pos[j + len] == pos[j] + len) ++len;
    if (r->n >= kMaxRuns) return false;
    r->src[r->n] = (int8_t)j;
    r->dst[r->n] = (int8_t)pos[j];
    r->len[r->n] = (int8_t)len;
    r->n++;
    j += len;
  }
  return true;
}

namespace {

int index_of(const std::vector<int>& v, int x) {
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i] == x) return (int)i;
  return -1;
}
bool contains(const std::vector<int>& v, int x) { return index_of(v, x) >= 0; }

// Position (bit weight) of layout entry i in a rank-r tensor: r - 1 - i.
int pos_in(const std::vector<int>& layout, int wire) {
  int i = index_of(layout, wire);
  return i < 0 ? -1 : (int)layout.size() - 1 - i;
}

// Reorders FP64 data from layout `from` to layout `to` (same wire set).
std::vector<cd> relayout(const std::vector<cd>& d, const std::vector<int>& from,
                         const std::vector<int>& to) {
  const int r = (int)from.size();
  std::vector<cd> out(d.size());
  std::vector<int> src_pos(r);  // for each target position, source position
  for (int i = 0; i < r; ++i) src_pos[r - 1 - i] = pos_in(from, to[i]);
  for (size_t t = 0; t < d.size(); ++t) {
    size_t s = 0;
    for (int q = 0; q < r; ++q)
      if (t >> q & 1) s |= (size_t)1 << src_pos[q];
    out[t] = d[s];
  }
  return out;
}

// Host contraction with sliced wires kept as batch indices (a shared sliced
// wire is not summed; both operands see the same fixed value in every slice).
HostTensor host_contract(const HostTensor& X, const HostTensor& Y, const std::vector<int>& slice_idx) {
  auto sliced = [&](int w) { return slice_idx[w] >= 0; };
  std::vector<int> zw, cw;
  for (int w : X.wires) {
    if (contains(Y.wires, w) && !sliced(w))
      cw.push_back(w);
    else
      zw.push_back(w);
  }
  for (int w : Y.wires)
    if (!contains(X.wires, w)) zw.push_back(w);
  const int rz = (int)zw.size(), rc = (int)cw.size();
  const size_t nz = (size_t)1 << rz, nc = (size_t)1 << rc;
  std::vector<size_t> xz(nz, 0), yz(nz, 0), xc(nc, 0), yc(nc, 0);
  const int rx = (int)X.wires.size(), ry = (int)Y.wires.size();
  for (int i = 0; i < rz; ++i) {
    int w = zw[i];
    int bit = rz - 1 - i;
    int px = pos_in(X.wires, w), py = pos_in(Y.wires, w);
    for (size_t z = 0; z < nz; ++z)
      if (z >> bit & 1) {
        if (px >= 0) xz[z] |= (size_t)1 << px;
        if (py >= 0) yz[z] |= (size_t)1 << py;
      }
  }
  for (int i = 0; i < rc; ++i) {
    int w = cw[i];
    int bit = rc - 1 - i;
    int px = pos_in(X.wires, w), py = pos_in(Y.wires, w);
    for (size_t c = 0; c < nc; ++c)
      if (c >> bit & 1) {
        xc[c] |= (size_t)1 << px;
        yc[c] |= (size_t)1 << py;
      }
  }
  (void)rx;
  (void)ry;
  HostTensor Z;
  Z.wires = zw;
  Z.data.assign(nz, cd(0, 0));
  for (size_t z = 0; z < nz; ++z) {
    cd acc(0, 0);
    for (size_t c = 0; c < nc; ++c) acc += X.data[xz[z] | xc[c]] * Y.data[yz[z] | yc[c]];
    Z.data[z] = acc;
  }
  return Z;
}

struct Buf {
  int64_t elems;
  int t0, t1;
  int64_t off = -1;
  int id;
};

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Greedy-by-size placement of buffers with time intervals [t0, t1].
int64_t place_buffers(std::vector<Buf>& bufs) {
  const int64_t A = 64;  // 512 B for complex64
  std::vector<int> order(bufs.size());
  for (size_t i = 0; i < bufs.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    if (bufs[a].elems != bufs[b].elems) return bufs[a].elems > bufs[b].elems;
    return a < b;
  });
  std::vector<int> placed;
  int64_t top = 0;
  for (int i : order) {
    Buf& b = bufs[i];
    std::vector<std::pair<int64_t, int64_t>> busy;
    for (int j : placed) {
      const Buf& o = bufs[j];
      if (o.t1 < b.t0 || b.t1 < o.t0) continue;
      busy.push_back({o.off, o.off + align_up(o.elems, A)});
    }
    std::sort(busy.begin(), busy.end());
    int64_t cand = 0;
    for (auto& iv : busy) {
      if (cand + align_up(b.elems, A) <= iv.first) break;
      cand = std::max(cand, iv.second);
    }
    b.off = cand;
    top = std::max(top, cand + align_up(b.elems, A));
    placed.push_back(i);
  }
  return top;
}

void json_runs(std::ostringstream& js, const Runs& r) {
  js << "[";
  for (int i = 0; i < r.n; ++i) js << (i ? "," : "") << "[" << (int)r.src[i] << "," << (int)r.dst[i] << "," << (int)r.len[i] << "]";
  js << "]";
}
void json_ref(std::ostringstream& js, const TRef& t) { js << "[" << t.region << "," << t.off << "]"; }
void json_vec(std::ostringstream& js, const std::vector<int>& v) {
  js << "[";
  for (size_t i = 0; i < v.size(); ++i) js << (i ? "," : "") << v[i];
  js << "]";
}

}  // namespace

// ---------------------------------------------------------------------------

static int build_network(PlanCore& P, std::vector<HostTensor>& leaves, std::string& err) {
  const int n = P.n_qubits;
  std::vector<int> open_sorted = P.open_q;
  std::sort(open_sorted.begin(), open_sorted.end());
  leaves.clear();
  for (int q = 0; q < n; ++q) {
    HostTensor t;
    t.wires = {q};
    t.data = {cd(1, 0), cd(0, 0)};
    leaves.push_back(t);
  }
  std::vector<int> cur(n);
  for (int q = 0; q < n; ++q) cur[q] = q;
  int nw = n;
  for (size_t g = 0; g < P.gates.size(); ++g) {
    const tn_gate& G = P.gates[g];
    HostTensor t;
    std::vector<int> ins, outs;
    for (int j = 0; j < G.nq; ++j) ins.push_back(cur[G.q[j]]);
    for (int j = 0; j < G.nq; ++j) {
      cur[G.q[j]] = nw;
      outs.push_back(nw++);
    }
    t.wires = outs;
    t.wires.insert(t.wires.end(), ins.begin(), ins.end());
    const int d = 1 << G.nq;
    t.data.resize((size_t)d * d);
    // tensor index (outs..., ins...) = row-major matrix index (row, col)
    for (int i = 0; i < d * d; ++i) t.data[i] = cd(G.m[2 * i], G.m[2 * i + 1]);
    leaves.push_back(t);
  }
  for (int q = 0; q < n; ++q) {
    if (std::binary_search(open_sorted.begin(), open_sorted.end(), q)) continue;
    HostTensor t;
    t.wires = {cur[q]};
    int b = P.out_bits.empty() ? 0 : (P.out_bits[q] & 1);
    t.data = {cd(b == 0 ? 1 : 0, 0), cd(b == 1 ? 1 : 0, 0)};
    leaves.push_back(t);
  }
  P.n_wires = nw;
  P.n_leaves = (int32_t)leaves.size();
  P.leaf_wires.clear();
  for (auto& l : leaves) P.leaf_wires.push_back(l.wires);
  P.open_wires.clear();
  for (int q : open_sorted) P.open_wires.push_back(cur[q]);
  (void)err;
  return TN_OK;
}

static int elem_bytes_plan(const PlanCore& P) { return P.opts.dtype == TN_DTYPE_C64 ? 8 : 4; }

static void add_stats_step(PlanCore& P, int nM, int nN, int nK, int ra, int rb, int rc) {
  const double eb = elem_bytes_plan(P);
  P.stats.flops_per_slice += 8.0 * std::ldexp(1.0, nM + nN + nK);
  P.stats.bytes_per_slice += eb * (std::ldexp(1.0, ra) + std::ldexp(1.0, rb) + std::ldexp(1.0, rc));
  if (nK < 64) P.stats.k_hist[nK]++;
}

void make_json(PlanCore& P) {
  const int L = P.n_leaves;
  std::ostringstream js;
  js << "{\"n_leaves\":" << L << ",\"n_wires\":" << P.n_wires << ",\"arena_elems\":" << P.arena_elems
     << ",\"leaves_elems\":" << P.leaves_elems << ",\"bound_elems\":" << P.bound_elems << ",\"open_wires\":";
  json_vec(js, P.open_wires);
  js << ",\"dev_leaves\":[";
  for (size_t i = 0; i < P.dev_leaves.size(); ++i) {
    auto& d = P.dev_leaves[i];
    js << (i ? "," : "") << "{\"ssa\":" << d.ssa << ",\"layout\":";
    json_vec(js, d.layout);
    js << ",\"n_sliced\":" << d.n_sliced << ",\"slice_bit\":";
    json_vec(js, d.slice_bit);
    js << ",\"stored_off\":" << d.stored_off << ",\"bound_off\":" << d.bound_off << "}";
  }
  js << "],\"binds\":[";
  for (size_t i = 0; i < P.binds.size(); ++i) {
    auto& b = P.binds[i];
    js << (i ? "," : "") << "{\"src\":" << b.src_off << ",\"dst\":" << b.dst_off << ",\"n\":" << b.n_elems
       << ",\"sbit\":[";
    for (int j = 0; j < b.n_sl; ++j) js << (j ? "," : "") << b.sbit[j];
    js << "],\"pos\":[";
    for (int j = 0; j < b.n_sl; ++j) js << (j ? "," : "") << b.pos[j];
    js << "]}";
  }
  js << "],\"ops\":[";
  for (size_t i = 0; i < P.ops.size(); ++i) {
    const Op& op = P.ops[i];
    js << (i ? "," : "") << "{\"kind\":" << op.kind << ",\"step\":" << op.step << ",\"flops\":" << op.flops
       << ",\"bytes\":" << op.bytes << ",\"a\":";
    json_ref(js, op.a);
    js << ",\"b\":";
    json_ref(js, op.b);
    js << ",\"c\":";
    json_ref(js, op.c);
    if (op.kind == kOpPermute) {
      js << ",\"rank\":" << op.perm.rank << ",\"perm\":[";
      for (int q = 0; q < op.perm.rank; ++q) js << (q ? "," : "") << op.perm.perm[q];
      js << "]";
    } else if (op.kind == kOpGemm) {
      js << ",\"M\":" << op.gemm.M << ",\"N\":" << op.gemm.N << ",\"K\":" << op.gemm.K << ",\"form\":" << op.gemm.form
         << ",\"split_k\":" << op.gemm.split_k << ",\"tile\":" << op.gemm.tile << ",\"split_max\":"
         << op.gemm.split_max << ",\"occ\":" << op.gemm.occ << ",\"ga\":" << op.gemm.gather_a
         << ",\"s_out\":" << op.s_out << ",\"w\":";
      json_ref(js, op.w);
      if (op.gemm.gather_a) {
        js << ",\"aM\":";
        json_runs(js, op.idx.aM);
        js << ",\"aK\":";
        json_runs(js, op.idx.aK);
      }
    } else {
      js << ",\"nM\":" << op.idx.nM << ",\"nN\":" << op.idx.nN << ",\"nK\":" << op.idx.nK << ",\"aM\":";
      json_runs(js, op.idx.aM);
      js << ",\"aK\":";
      json_runs(js, op.idx.aK);
      js << ",\"bN\":";
      json_runs(js, op.idx.bN);
      js << ",\"bK\":";
      json_runs(js, op.idx.bK);
      js << ",\"tM\":" << op.idx.tM << ",\"tK\":" << op.idx.tK << ",\"s_out\":" << op.s_out << ",\"w\":";
      json_ref(js, op.w);
    }
    js << "}";
  }
  js << "],\"steps\":[";
  for (size_t i = 0; i < P.steps.size(); ++i) {
    const PlanCore::StepInfo& st = P.steps[i];
    js << (i ? "," : "") << "{\"t\":" << st.t << ",\"nM\":" << st.nM << ",\"nN\":" << st.nN << ",\"nK\":" << st.nK
       << ",\"cls\":" << st.cls << ",\"key\":\"" << st.key << "\",\"tuned\":" << (P.class_override.count(st.t) ? "true" : "false") << "}";
  }
  js << "],\"accum\":{\"n_open\":" << P.accum.n_open << ",\"root\":";
  json_ref(js, P.accum.root);
  js << ",\"y2root\":";
  json_runs(js, P.accum.y2root);
  js << std::setprecision(17) << ",\"root_scale\":" << P.accum.root_scale << ",\"rounding_factor\":["
     << P.accum.kappa0_re << "," << P.accum.kappa0_im << "]}}";
  P.json = js.str();
}

static int build_pair_network(PlanCore& P, std::vector<HostTensor>& leaves, std::string& err) {
  leaves.assign(2, HostTensor{});
  leaves[0].wires = P.pair_a;
  leaves[1].wires = P.pair_b;
  int mx = -1;
  for (const auto* v : {&P.pair_a, &P.pair_b, &P.pair_out})
    for (int w : *v) {
      if (w < 0 || w > 4095) {
        err = "index label out of range";
        return TN_E_ARG;
      }
      mx = std::max(mx, w);
    }
  for (const auto* v : {&P.pair_a, &P.pair_b}) {
    std::vector<int> t = *v;
    std::sort(t.begin(), t.end());
    if (std::adjacent_find(t.begin(), t.end()) != t.end()) {
      err = "repeated index label within one tensor";
      return TN_E_ARG;
    }
  }
  std::vector<int> expect;
  for (int w : P.pair_a)
    if (!contains(P.pair_b, w)) expect.push_back(w);
  for (int w : P.pair_b)
    if (!contains(P.pair_a, w)) expect.push_back(w);
  std::vector<int> got = P.pair_out;
  std::sort(expect.begin(), expect.end());
  std::sort(got.begin(), got.end());
  if (expect != got) {
    err = "output labels must be exactly the labels of A and B that are not shared";
    return TN_E_TOPOLOGY;
  }
  P.n_wires = mx + 1;
  P.n_leaves = 2;
  P.leaf_wires = {P.pair_a, P.pair_b};
  P.open_wires = P.pair_out;
  P.pairs = {0, 1};
  P.sliced.clear();
  return TN_OK;
}

static PlanCore::StepInfo step_info(int t, const std::vector<int>& La, const std::vector<int>& Lb,
                                    const std::vector<int>& Lc, int nM, int nN, int nK, int cls) {
  PlanCore::StepInfo st;
  st.t = t;
  st.nM = nM;
  st.nN = nN;
  st.nK = nK;
  st.cls = cls;
  std::map<int, int> lab;
  auto relabel = [&](const std::vector<int>& in, std::vector<int>& out) {
    for (int w : in) {
      auto it = lab.find(w);
      if (it == lab.end()) it = lab.emplace(w, (int)lab.size()).first;
      out.push_back(it->second);
    }
    if (!st.key.empty()) st.key += '/';
    for (size_t i = 0; i < out.size(); ++i) st.key += (i ? "." : "") + std::to_string(out[i]);
  };
  relabel(La, st.la);
  relabel(Lb, st.lb);
  relabel(Lc, st.lc);
  return st;
}

int build_plan(PlanCore& P, std::string& err) {
  const int n = P.n_qubits;
  std::vector<HostTensor> leaves;
  int rc = P.pair_mode ? build_pair_network(P, leaves, err) : build_network(P, leaves, err);
  if (rc) return rc;
  const int L = P.n_leaves;
  const int S = (int)P.pairs.size() / 2;
  if (S != L - 1) {
    err = "order has " + std::to_string(S) + " steps; a full tree over " + std::to_string(L) +
          " leaves needs " + std::to_string(L - 1);
    return TN_E_TOPOLOGY;
  }
  // sliced wires
  P.wire_slice_idx.assign(P.n_wires, -1);
  for (size_t j = 0; j < P.sliced.size(); ++j) {
    int w = P.sliced[j];
    if (w < 0 || w >= P.n_wires) {
      err = "sliced wire " + std::to_string(w) + " out of range";
      return TN_E_TOPOLOGY;
    }
    if (P.wire_slice_idx[w] >= 0) {
      err = "sliced wire " + std::to_string(w) + " listed twice";
      return TN_E_ARG;
    }
    if (contains(P.open_wires, w)) {
      err = "sliced wire " + std::to_string(w) + " is an open output wire";
      return TN_E_ARG;
    }
    P.wire_slice_idx[w] = (int)j;
  }
  // SSA validation and host wire sets (sliced wires kept as batch indices)
  std::vector<std::vector<int>> hw(L + S);
  for (int i = 0; i < L; ++i) hw[i] = P.leaf_wires[i];
  std::vector<int> consumer(L + S, -1);
  for (int t = 0; t < S; ++t) {
    int a = P.pairs[2 * t], b = P.pairs[2 * t + 1];
    for (int x : {a, b}) {
      if (x < 0 || x >= L + t) {
        err = "step " + std::to_string(t) + " names id " + std::to_string(x) + " not yet defined";
        return TN_E_TOPOLOGY;
      }
      if (consumer[x] >= 0) {
        err = "id " + std::to_string(x) + " consumed twice (steps " + std::to_string(consumer[x]) + ", " +
              std::to_string(t) + ")";
        return TN_E_TOPOLOGY;
      }
      consumer[x] = t;
    }
    if (a == b) {
      err = "step " + std::to_string(t) + " contracts an id with itself";
      return TN_E_TOPOLOGY;
    }
    std::vector<int> z;
    for (int w : hw[a])
      if (!(contains(hw[b], w) && P.wire_slice_idx[w] < 0)) z.push_back(w);
    for (int w : hw[b])
      if (!contains(hw[a], w)) z.push_back(w);
    hw[L + t] = z;
  }
  const int root = L + S - 1;
  {
    // the root must carry exactly the open wires (sliced wires dropped)
    std::vector<int> rw;
    for (int w : hw[root])
      if (P.wire_slice_idx[w] < 0) rw.push_back(w);
    std::vector<int> a = rw, b = P.open_wires;
    std::sort(a.begin(), a.end());
    std::sort(b.begin(), b.end());
    if (a != b) {
      err = "the contraction does not end on the open wires (disconnected order or dangling wires)";
      return TN_E_TOPOLOGY;
    }
  }
  // host / device split
  P.on_host.assign(L + S, false);
  for (int i = 0; i < L; ++i) P.on_host[i] = true;
  std::vector<HostTensor> ht(L + S);
  for (int i = 0; i < L; ++i) ht[i] = leaves[i];
  P.n_host_steps = 0;
  const int fold = P.opts.host_fold_log2;
  for (int t = 0; t < S; ++t) {
    int a = P.pairs[2 * t], b = P.pairs[2 * t + 1];
    bool host = P.on_host[a] && P.on_host[b] && (t != S - 1) && (int)hw[L + t].size() <= fold;
    if (host) {
      std::set<int> u(hw[a].begin(), hw[a].end());
      u.insert(hw[b].begin(), hw[b].end());
      host = (int)u.size() <= 22;
    }
    if (host) {
      ht[L + t] = host_contract(ht[a], ht[b], P.wire_slice_idx);
      P.on_host[L + t] = true;
      P.n_host_steps++;
      ht[a].data.clear();
      ht[b].data.clear();
    }
  }
  // device leaves: host tensors consumed by device steps (or the root itself)
  P.dev_leaves.clear();
  std::map<int, int> devleaf_of;  // ssa -> index
  auto add_devleaf = [&](int ssa) {
    if (devleaf_of.count(ssa)) return;
    DevLeaf d;
    d.ssa = ssa;
    std::vector<std::pair<int, int>> sl;
    std::vector<int> rest;
    for (int w : ht[ssa].wires) {
      if (P.wire_slice_idx[w] >= 0)
        sl.push_back({P.wire_slice_idx[w], w});
      else
        rest.push_back(w);
    }
    std::sort(sl.begin(), sl.end());
    if (sl.size() > 8) return;  // reported below
    for (auto& p : sl) {
      d.layout.push_back(p.second);
      d.slice_bit.push_back(p.first);
    }
    d.n_sliced = (int)sl.size();
    d.layout.insert(d.layout.end(), rest.begin(), rest.end());
    if (!P.pair_mode) d.data = relayout(ht[ssa].data, ht[ssa].wires, d.layout);
    devleaf_of[ssa] = (int)P.dev_leaves.size();
    P.dev_leaves.push_back(std::move(d));
  };
  if (S == 0) {
    add_devleaf(root);
    P.root_is_leaf = 1;
  } else {
    P.root_is_leaf = 0;
    for (int t = 0; t < S; ++t) {
      if (P.on_host[L + t]) continue;
      for (int x : {P.pairs[2 * t], P.pairs[2 * t + 1]})
        if (P.on_host[x]) {
          add_devleaf(x);
          if (!devleaf_of.count(x)) {
            err = "a folded leaf carries more than 8 sliced wires";
            return TN_E_UNSUPPORTED;
          }
        }
    }
  }
  // leaves region and bind descriptors
  P.leaves_elems = 0;
  P.bound_elems = 0;
  P.binds.clear();
  for (auto& d : P.dev_leaves) {
    int64_t ne = P.pair_mode ? 0 : (int64_t)d.data.size();
    d.stored_off = P.leaves_elems;
    P.leaves_elems += align_up(ne, 64);
    if (d.n_sliced > 0) {
      int64_t nb = ne >> d.n_sliced;
      d.bound_off = P.bound_elems;
      P.bound_elems += align_up(nb, 64);
      BindDesc bd{};
      bd.src_off = d.stored_off;
      bd.dst_off = d.bound_off;
      bd.n_elems = nb;
      bd.n_sl = d.n_sliced;
      const int r = (int)d.layout.size();
      for (int i = 0; i < d.n_sliced; ++i) {
        bd.sbit[i] = d.slice_bit[i];
        bd.pos[i] = r - 1 - i;
      }
      P.binds.push_back(bd);
    }
  }
  // device steps
  std::vector<std::vector<int>> lay(L + S);  // device layout per ssa (sliced wires removed)
  std::vector<TRef> where(L + S);
  for (auto& d : P.dev_leaves) {
    lay[d.ssa] = std::vector<int>(d.layout.begin() + d.n_sliced, d.layout.end());
    if (P.pair_mode)
      where[d.ssa] = TRef{d.ssa == 0 ? kExtA : kExtB, 0};
    else if (d.n_sliced > 0)
      where[d.ssa] = TRef{kBound, d.bound_off};
    else
      where[d.ssa] = TRef{kLeaves, d.stored_off};
  }
  P.ops.clear();
  P.steps.clear();
  P.n_slots = 0;
  std::vector<Buf> bufs;
  std::vector<int> buf_of_ssa(L + S, -1);
  struct Pending {
    int op, which, buf;
  };
  std::vector<Pending> fix;  // op operand -> buffer id (resolved after placement)
  int dstep = 0;
  int max_log2 = 0;
  std::memset(P.stats.k_hist, 0, sizeof(P.stats.k_hist));
  P.stats.flops_per_slice = P.stats.bytes_per_slice = P.stats.moved_per_slice = 0;
  P.stats.n_dense = P.stats.n_skinny = P.stats.n_generic = P.stats.n_permute = 0;
  std::vector<int> step_time(S, -1);
  for (int t = 0; t < S; ++t) {
    if (P.on_host[L + t]) continue;
    step_time[t] = dstep;
    int x = P.pairs[2 * t], y = P.pairs[2 * t + 1];
    const std::vector<int>& Lx = lay[x];
    const std::vector<int>& Ly = lay[y];
    int ia = x, ib = y;
    if (Ly.size() > Lx.size()) std::swap(ia, ib);
    const std::vector<int>& La = lay[ia];
    const std::vector<int>& Lb = lay[ib];
    std::vector<int> K, MA, NB;
    for (int w : La) (contains(Lb, w) ? K : MA).push_back(w);
    for (int w : Lb)
      if (!contains(La, w)) NB.push_back(w);
    const int nM = (int)MA.size(), nN = (int)NB.size(), nK = (int)K.size();
    const int ra = (int)La.size(), rb = (int)Lb.size(), rcn = nM + nN;
    max_log2 = std::max({max_log2, ra, rb, rcn});
    if (rcn > kMaxRank || ra > kMaxRank || rb > kMaxRank) {
      err = "tensor rank above " + std::to_string(kMaxRank);
      return TN_E_UNSUPPORTED;
    }
    add_stats_step(P, nM, nN, nK, ra, rb, rcn);
    std::vector<int> Lc = MA;
    Lc.insert(Lc.end(), NB.begin(), NB.end());
    lay[L + t] = Lc;
    // result buffer
    Buf cb{(int64_t)1 << rcn, dstep, dstep, -1, (int)bufs.size()};
    int cbuf = (int)bufs.size();
    bufs.push_back(cb);
    buf_of_ssa[L + t] = cbuf;
    // extend lifetimes of operand buffers to this step
    for (int o : {ia, ib})
      if (buf_of_ssa[o] >= 0) bufs[buf_of_ssa[o]].t1 = dstep;

    auto operand_ref = [&](int ssa, int op, int which) {
      if (buf_of_ssa[ssa] >= 0) fix.push_back({op, which, buf_of_ssa[ssa]});
      return where[ssa];
    };

    const bool half = P.opts.dtype != TN_DTYPE_C64;
    const double eb = elem_bytes_plan(P);
    const int64_t f2 = 8 / (int64_t)eb;  // plan elements per float2 workspace entry
    // kernel class: the planner's rule, unless the class autotuner measured
    // another valid class to be faster for this step
    const unsigned valid = step_classes(nM, nN, nK);
    int cls = default_class(nM, nN, nK);
    {
      auto ov = P.class_override.find(t);
      if (ov != P.class_override.end() && ov->second >= 0 && ov->second < 32 && (valid & (1u << ov->second)))
        cls = ov->second;
    }
    P.steps.push_back(step_info(t, La, Lb, Lc, nM, nN, nK, cls));
    if (cls == kOpGemm) {
      // K order: keep whichever operand already has K as its lowest block
      auto k_low_block = [&](const std::vector<int>& Lx2, std::vector<int>& kord) {
        int r = (int)Lx2.size();
        if (r < nK) return false;
        std::vector<int> tail(Lx2.end() - nK, Lx2.end());
        std::vector<int> s1 = tail, s2 = K;
        std::sort(s1.begin(), s1.end());
        std::sort(s2.begin(), s2.end());
        if (s1 != s2) return false;
        kord = tail;
        return true;
      };
      std::vector<int> Kord;
      if (!k_low_block(La, Kord) && !k_low_block(Lb, Kord)) Kord = K;
      // a large A that would need a permute is read in place by the GEMM,
      // with the K bits in A's own order (B is permuted to match), for sums
      // of 2^kGatherMinK terms or more.  Scaled storage uses the 4M form
      // there.
      IndexOp gidx;
      bool gather = false;
      {
        std::vector<int> wa = MA;
        wa.insert(wa.end(), Kord.begin(), Kord.end());
        // the in-place kernels have no K split: a long sum needs enough
        // 128x128 output tiles (512, two per CU) on its own
        const bool fills = nM + nN - 14 >= 9 || nK < 11;
        if (wa != La && ra >= kGatherMinLog2 && nK >= kGatherMinK && fills &&
            (!half || P.opts.gemm_form != TN_GEMM_3M)) {
          gidx.nM = nM;
          gidx.nN = nN;
          gidx.nK = nK;
          std::vector<int> p;
          for (int i = 0; i < nM; ++i) p.push_back(pos_in(La, MA[nM - 1 - i]));
          bool ok = make_runs(p, &gidx.aM);
          p.clear();
          for (int i = 0; i < nK; ++i) p.push_back(pos_in(La, K[nK - 1 - i]));
          ok = ok && make_runs(p, &gidx.aK);
          if (ok && gemm_gather_ok(gidx)) {
            gather = true;
            Kord = K;
          }
        }
      }
      std::vector<int> wantA = MA, wantB = NB;
      wantA.insert(wantA.end(), Kord.begin(), Kord.end());
      wantB.insert(wantB.end(), Kord.begin(), Kord.end());
      TRef aref, bref;
      int a_tmp = -1, b_tmp = -1;
      for (int side = 0; side < 2; ++side) {
        const std::vector<int>& have = side ? Lb : La;
        const std::vector<int>& want = side ? wantB : wantA;
        int ssa = side ? ib : ia;
        if (have == want || (side == 0 && gather)) continue;
        Op op;
        op.kind = kOpPermute;
        op.step = t;
        int r = (int)have.size();
        op.perm.rank = r;
        for (int q = 0; q < r; ++q) op.perm.perm[q] = pos_in(have, want[r - 1 - q]);
        int opi = (int)P.ops.size();
        op.a = operand_ref(ssa, opi, 0);
        Buf tb{(int64_t)1 << r, dstep, dstep, -1, (int)bufs.size()};
        int tbi = (int)bufs.size();
        bufs.push_back(tb);
        fix.push_back({opi, 2, tbi});
        op.bytes = 2.0 * eb * std::ldexp(1.0, r);
        P.ops.push_back(op);
        P.stats.n_permute++;
        if (side)
          b_tmp = tbi;
        else
          a_tmp = tbi;
      }
      Op g;
      g.kind = kOpGemm;
      g.step = t;
      g.gemm.M = (int64_t)1 << nM;
      g.gemm.N = (int64_t)1 << nN;
      g.gemm.K = (int64_t)1 << nK;
      // auto: on FP32 matrix cores the 3M form (three real products per
      // complex product) is the faster one on every compute-bound shape
      // measured; on FP16/BF16 cores 4M is (3M's third operand plane makes
      // those kernels bound by LDS bandwidth)
      g.gemm.form = P.opts.gemm_form != TN_GEMM_AUTO ? P.opts.gemm_form : (half ? TN_GEMM_4M : TN_GEMM_3M);
      int gi = (int)P.ops.size();
      if (gather) {
        g.gemm.gather_a = 1;
        g.gemm.tile = 128;
        g.idx = gidx;
      }
      // split K when the output has too few tiles (128x128, or 64x64 when an
      // extent is 64) to fill the chip
      if (nM >= 6 && nN >= 6 && !gather) {
        const int tl = (nM >= 7 && nN >= 7) ? 7 : 6;
        const int64_t tiles = (int64_t)1 << (nM - tl + nN - tl);
        int sp = 1;
        while (tiles * sp < 2048 && ((int64_t)1 << nK) / (sp * 2) >= 1024 && sp < 64 &&
               ((int64_t)sp * 2 << (nM + nN)) <= ((int64_t)1 << 28))
          sp *= 2;
        // with tuning, room for every split the tuner may try: slabs of at
        // least 256 along K, at most 64 slabs, workspace <= 2^28 entries,
        // and only while the output has fewer than 8192 64x64 tiles
        int cap = sp;
        if (P.opts.tune && ((int64_t)1 << (nM + nN - 12)) < 8192)
          while (cap < 64 && ((int64_t)1 << nK) / (cap * 2) >= 256 &&
                 ((int64_t)cap * 2 << (nM + nN)) <= ((int64_t)1 << 28))
            cap *= 2;
        g.gemm.split_k = sp;
        g.gemm.split_max = cap;
        if (cap > 1) {
          Buf wb{((int64_t)cap << (nM + nN)) * f2, dstep, dstep, -1, (int)bufs.size()};
          fix.push_back({gi, 3, (int)bufs.size()});
          bufs.push_back(wb);
        }
      }
      if (a_tmp >= 0)
        fix.push_back({gi, 0, a_tmp});
      else
        aref = operand_ref(ia, gi, 0);
      if (b_tmp >= 0)
        fix.push_back({gi, 1, b_tmp});
      else
        bref = operand_ref(ib, gi, 1);
      g.a = aref;
      g.b = bref;
      fix.push_back({gi, 2, cbuf});
      g.flops = 8.0 * std::ldexp(1.0, nM + nN + nK);
      g.bytes = eb * (std::ldexp(1.0, ra) + std::ldexp(1.0, rb) + std::ldexp(1.0, rcn));
      g.ssa_a = ia;
      g.ssa_b = ib;
      g.ssa_c = L + t;
      if (half) g.max_slot = P.n_slots++;
      P.ops.push_back(g);
      P.stats.n_dense++;
    } else {
      Op g;
      const bool splitk = cls == kOpSplitK;
      const bool skinny = cls == kOpSkinny;
      g.kind = cls;
      g.step = t;
      g.idx.nM = nM;
      g.idx.nN = nN;
      g.idx.nK = nK;
      // split-K into more than 8 x 8 outputs: consecutive threads take
      // consecutive k, so an operand whose lowest k bits are not its lowest
      // bits (in order) is gathered across the whole tensor; such an operand
      // (of 2^12 entries or more) is first permuted to [free wires, K]
      int tmp[2] = {-1, -1};
      std::vector<int> lay2[2] = {La, Lb};
      // the matrix-core skewed kernel with a long sum stages B chunk by
      // chunk: a B whose low k bits are scattered is permuted first too
      // (B only; A is read in place)
      const bool skew_long = cls == kOpSkew && nK >= 7;
      if ((splitk && !splitk_chunk_ok(nM, nN, nK)) || skew_long) {
        for (int side = skew_long ? 1 : 0; side < 2; ++side) {
          const std::vector<int>& have = side ? Lb : La;
          const int r = (int)have.size();
          bool aligned = true;
          for (int i = 0; i < std::min(nK, 8); ++i) aligned &= pos_in(have, K[nK - 1 - i]) == i;
          if (aligned || r < 12) continue;
          std::vector<int> want = side ? NB : MA;
          want.insert(want.end(), K.begin(), K.end());
          Op op;
          op.kind = kOpPermute;
          op.step = t;
          op.perm.rank = r;
          for (int q = 0; q < r; ++q) op.perm.perm[q] = pos_in(have, want[r - 1 - q]);
          const int opi = (int)P.ops.size();
          op.a = operand_ref(side ? ib : ia, opi, 0);
          Buf tb{(int64_t)1 << r, dstep, dstep, -1, (int)bufs.size()};
          tmp[side] = (int)bufs.size();
          bufs.push_back(tb);
          fix.push_back({opi, 2, tmp[side]});
          op.bytes = 2.0 * eb * std::ldexp(1.0, r);
          P.ops.push_back(op);
          P.stats.n_permute++;
          lay2[side] = want;
        }
      }
      const std::vector<int>& LA = lay2[0];
      const std::vector<int>& LB = lay2[1];
      std::vector<int> p;
      bool ok = true;
      p.clear();
      for (int i = 0; i < nM; ++i) p.push_back(pos_in(LA, MA[nM - 1 - i]));
      ok &= make_runs(p, &g.idx.aM);
      p.clear();
      for (int i = 0; i < nK; ++i) p.push_back(pos_in(LA, K[nK - 1 - i]));
      ok &= make_runs(p, &g.idx.aK);
      p.clear();
      for (int i = 0; i < nN; ++i) p.push_back(pos_in(LB, NB[nN - 1 - i]));
      ok &= make_runs(p, &g.idx.bN);
      p.clear();
      for (int i = 0; i < nK; ++i) p.push_back(pos_in(LB, K[nK - 1 - i]));
      ok &= make_runs(p, &g.idx.bK);
      if (!ok) {
        err = "index map too fragmented";
        return TN_E_UNSUPPORTED;
      }
      int gi = (int)P.ops.size();
      if (tmp[0] >= 0)
        fix.push_back({gi, 0, tmp[0]});
      else
        g.a = operand_ref(ia, gi, 0);
      if (tmp[1] >= 0)
        fix.push_back({gi, 1, tmp[1]});
      else
        g.b = operand_ref(ib, gi, 1);
      fix.push_back({gi, 2, cbuf});
      if (splitk) {
        Buf wb{(splitk_grid(nK) << (nM + nN)) * f2, dstep, dstep, -1, (int)bufs.size()};
        fix.push_back({gi, 3, (int)bufs.size()});
        bufs.push_back(wb);
      }
      g.flops = 8.0 * std::ldexp(1.0, nM + nN + nK);
      g.bytes = eb * (std::ldexp(1.0, ra) + std::ldexp(1.0, rb) + std::ldexp(1.0, rcn));
      g.ssa_a = ia;
      g.ssa_b = ib;
      g.ssa_c = L + t;
      if (half) g.max_slot = P.n_slots++;
      P.ops.push_back(g);
      if (skinny || cls == kOpSkew)
        P.stats.n_skinny++;
      else
        P.stats.n_generic++;
    }
    dstep++;
  }
  // arena placement
  P.arena_elems = place_buffers(bufs);
  for (auto& f : fix) {
    Op& op = P.ops[f.op];
    TRef r{kArena, bufs[f.buf].off};
    if (f.which == 0)
      op.a = r;
    else if (f.which == 1)
      op.b = r;
    else if (f.which == 2)
      op.c = r;
    else
      op.w = r;
  }
  for (auto& op : P.ops) P.stats.moved_per_slice += op.bytes;
  // final accumulation
  P.accum = AccumDesc{};
  P.accum.n_open = (int)P.open_wires.size();
  P.root_layout = lay[root];
  {
    const std::vector<int>& Lr = lay[root];
    std::vector<int> p;
    for (int i = 0; i < P.accum.n_open; ++i) p.push_back(pos_in(Lr, P.open_wires[P.accum.n_open - 1 - i]));
    if (!make_runs(p, &P.accum.y2root)) {
      err = "output map too fragmented";
      return TN_E_UNSUPPORTED;
    }
    P.accum.root_ssa = root;
    if (P.root_is_leaf)
      P.accum.root = where[root];
    else
      P.accum.root = TRef{kArena, bufs[buf_of_ssa[root]].off};
  }
  if (P.opts.max_log2 > 0 && max_log2 > P.opts.max_log2) {
    err = "a per-slice tensor has 2^" + std::to_string(max_log2) + " entries, above the bound 2^" +
          std::to_string(P.opts.max_log2);
    return TN_E_MEM;
  }
  // stats
  tn_plan_stats& st = P.stats;
  st.n_slices = (int64_t)1 << P.sliced.size();
  st.n_leaves = L;
  st.n_host_steps = P.n_host_steps;
  st.n_device_steps = dstep;
  st.n_kernels = (int)P.ops.size() + 1 + (P.binds.empty() ? 0 : 1);
  st.max_log2 = max_log2;
  st.n_open = (int)P.open_wires.size();
  st.arena_bytes = P.arena_elems * elem_bytes_plan(P);
  st.leaf_bytes = (P.leaves_elems + P.bound_elems) * elem_bytes_plan(P);
  make_json(P);
  (void)n;
  return TN_OK;
}

void leaf_exponents(PlanCore& P) {
  for (DevLeaf& d : P.dev_leaves) {
    double mx = 0;
    for (const cd& v : d.data) mx = std::max({mx, std::fabs(v.real()), std::fabs(v.imag())});
    d.e = mx > 0 ? (int)std::ceil(std::log2(mx)) - kTargetLog2 : 0;
  }
}

void set_output_shift(Op& op, float max_acc) {
  int s = 0;
  if (max_acc > 0 && std::isfinite(max_acc)) s = (int)std::ceil(std::log2((double)max_acc)) - kTargetLog2;
  op.s_out = s;
  const float sc = (float)std::ldexp(1.0, -s);
  op.gemm.out_scale = sc;
  op.idx.out_scale = sc;
}

void propagate_exponents(PlanCore& P) {
  std::map<int, int> e;
  for (const DevLeaf& d : P.dev_leaves) e[d.ssa] = P.opts.dtype == TN_DTYPE_C64 ? 0 : d.e;
  for (const Op& op : P.ops)
    if (op.ssa_c >= 0) e[op.ssa_c] = e[op.ssa_a] + e[op.ssa_b] + op.s_out;
  P.accum.root_scale = std::ldexp(1.0, e.count(P.accum.root_ssa) ? e[P.accum.root_ssa] : 0);
}

int build_pair_plan(PlanCore& P, std::string& err) {
  P.pair_mode = true;
  P.opts.host_fold_log2 = 0;
  int rc = build_plan(P, err);
  if (rc) return rc;
  // the op that wrote the root
  int last = -1;
  for (int i = 0; i < (int)P.ops.size(); ++i)
    if (P.ops[i].c.region == kArena && P.ops[i].c.off == P.accum.root.off && P.ops[i].kind != kOpPermute) last = i;
  if (last < 0) {
    err = "internal: pair plan without a producing op";
    return TN_E_UNSUPPORTED;
  }
  if (P.root_layout == P.pair_out) {
    P.ops[last].c = TRef{kExtC, 0};
  } else {
    Op op;
    op.kind = kOpPermute;
    op.step = 0;
    const int r = (int)P.pair_out.size();
    op.perm.rank = r;
    for (int q = 0; q < r; ++q) op.perm.perm[q] = pos_in(P.root_layout, P.pair_out[r - 1 - q]);
    op.a = P.accum.root;
    op.c = TRef{kExtC, 0};
    op.bytes = 2.0 * elem_bytes_plan(P) * std::ldexp(1.0, r);
    P.ops.push_back(op);
    P.stats.n_permute++;
    P.stats.moved_per_slice += op.bytes;
  }
  P.stats.n_kernels = (int)P.ops.size();
  make_json(P);
  return TN_OK;
}

int refold_leaves(PlanCore& P, std::string& err) {
  // Re-run the whole host side with the new output bits; the device
  // structure (layouts, ops, offsets) does not depend on bit values.
  PlanCore Q = P;
  int rc = build_plan(Q, err);
  if (rc) return rc;
  if (Q.dev_leaves.size() != P.dev_leaves.size()) {
    err = "internal: refold changed the leaf structure";
    return TN_E_UNSUPPORTED;
  }
  for (size_t i = 0; i < P.dev_leaves.size(); ++i) P.dev_leaves[i].data = std::move(Q.dev_leaves[i].data);
  return TN_OK;
}

}  // namespace tnrcs

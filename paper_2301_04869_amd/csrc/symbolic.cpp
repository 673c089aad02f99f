// Host-side symbolic analysis: variable maps, fixed sparsity patterns, gather
// lists, fill-reducing ordering and the filled LU pattern of G_x.
#include "symbolic.h"

#include <algorithm>
#include <array>
#include <cstdio>
#include <limits>
#include <map>
#include <numeric>
#include <queue>
#include <set>
#include <tuple>
#include <utility>

namespace rkkt {
namespace {

struct Contrib {
  std::vector<int> src;
  double c = 0.0;
};
using SparseRow = std::map<int, Contrib>;  // internal z var -> contributions

struct KEntry {
  std::vector<int> wsrc;                          // LH sources
  std::vector<std::array<int, 2>> wprod;          // product of two H values
  std::vector<double> wcoef;
  double wconst = 0.0;
  std::vector<std::array<int, 3>> trip;           // (h row, H value a, H value b)
};

// Minimum-degree elimination on an undirected graph.  Returns the elimination
// order; fill[v] receives the neighbours of v that are still uneliminated when v
// is eliminated (the off-diagonal pattern of column v of the Cholesky-like
// factor of the symmetrised matrix).  Ties go to the smaller index.
std::vector<int> minimum_degree(int n, std::vector<std::vector<int>> adj,
                                std::vector<std::vector<int>>& fill) {
  std::set<std::pair<int, int>> pq;
  for (int v = 0; v < n; ++v) pq.insert({(int)adj[v].size(), v});
  std::vector<int> order;
  order.reserve(n);
  fill.assign(n, {});
  std::vector<int> merged;
  while (!pq.empty()) {
    int v = pq.begin()->second;
    pq.erase(pq.begin());
    order.push_back(v);
    const std::vector<int>& nv = adj[v];
    fill[v] = nv;
    for (int w : nv) {
      pq.erase({(int)adj[w].size(), w});
      merged.clear();
      std::set_union(adj[w].begin(), adj[w].end(), nv.begin(), nv.end(),
                     std::back_inserter(merged));
      std::vector<int> out;
      out.reserve(merged.size());
      for (int q : merged)
        if (q != v && q != w) out.push_back(q);
      adj[w].swap(out);
      pq.insert({(int)adj[w].size(), w});
    }
    adj[v].clear();
    adj[v].shrink_to_fit();
  }
  return order;
}

int find_pos(const std::vector<int>& ptr, const std::vector<int>& col, int row, int c) {
  auto b = col.begin() + ptr[row], e = col.begin() + ptr[row + 1];
  auto it = std::lower_bound(b, e, c);
  if (it == e || *it != c) return -1;
  return (int)(it - col.begin());
}


// Assigns the tasks of one phase to S slots, longest first to the least
// loaded slot (ties to the lowest slot), and returns each slot's task list.
void assign_tasks(const std::vector<long long>& cost, int S, std::vector<std::vector<int>>& slot_tasks) {
  std::vector<int> order(cost.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  for (auto& v : slot_tasks) v.clear();
  using Item = std::pair<long long, int>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int t = 0; t < S; ++t) heap.push({0, t});
  for (int t : order) {
    Item it = heap.top();
    heap.pop();
    slot_tasks[it.second].push_back(t);
    heap.push({it.first + cost[t], it.second});
  }
}

// Sources of the level-sliced pulls of one direction: for every row j, the
// rows i that read it, with the position of (i, j).  Up: (i, j) in the strict
// lower part (j < i); down: in the strict upper part (j > i).
std::vector<std::vector<std::pair<int, int>>> dependents(const Sym& s, bool up) {
  std::vector<std::vector<std::pair<int, int>>> dep(s.nx);
  for (int i = 0; i < s.nx; ++i) {
    const int e0 = up ? s.f_ptr[i] : s.f_diag[i] + 1;
    const int e1 = up ? s.f_diag[i] : s.f_ptr[i + 1];
    for (int e = e0; e < e1; ++e) dep[s.f_col[e]].push_back({i, e});
  }
  return dep;
}

// Source groups of the phases of one direction, for a chain of the last t
// rows.  Up: the rows before the chain of every level (the chain's rows are
// solved after the phases, in registers).  Down: the chain rows as one group
// (final once the chain is solved first), then the rows before the chain of
// every level.  Groups whose rows have no dependents outside the chain are
// dropped.
std::vector<std::vector<int>> phase_groups_t(const Sym& s, bool up, int t) {
  const std::vector<int>& lv_ptr = up ? s.lvu_ptr : s.lvd_ptr;
  const std::vector<int>& lv_rows = up ? s.lvu_rows : s.lvd_rows;
  const int nlev = (int)lv_ptr.size() - 1, c0 = s.nx - t;
  auto has_dep = [&](int j) {  // j has a dependent that is not a chain-internal pair
    const bool jc = j >= c0;
    if (up) {
      // dependents of j: rows i > j with (i, j) in L, i.e. (j, i) in U
      for (int e = s.f_diag[j] + 1; e < s.f_ptr[j + 1]; ++e)
        if (!(jc && s.f_col[e] >= c0)) return true;
    } else {
      for (int e = s.f_ptr[j]; e < s.f_diag[j]; ++e)
        if (!(jc && s.f_col[e] >= c0)) return true;
    }
    return false;
  };
  std::vector<std::vector<int>> g;
  if (!up && t > 0) {
    g.emplace_back();
    for (int i = c0; i < s.nx; ++i) g.back().push_back(i);
  }
  for (int q = 0; q < nlev; ++q) {
    std::vector<int> rows;
    bool any = false;
    for (int r = lv_ptr[q]; r < lv_ptr[q + 1]; ++r) {
      const int i = lv_rows[r];
      if (i < c0) {
        rows.push_back(i);
        any = any || has_dep(i);
      }
    }
    if (any) g.push_back(rows);
  }
  return g;
}

std::vector<std::vector<int>> phase_groups(const Sym& s, bool up) { return phase_groups_t(s, up, s.chain_t); }

// Tasks of one phase: (dest, source, position) sorted by dest then source,
// split into runs of one dest.  Pairs inside the chain are left to the chain
// solve.
void phase_tasks(const Sym& s, const std::vector<std::vector<std::pair<int, int>>>& dep,
                 const std::vector<int>& sources, std::vector<std::array<int, 3>>& items,
                 std::vector<std::pair<int, int>>& tasks) {
  items.clear();
  tasks.clear();
  const int c0 = s.nx - s.chain_t;
  for (int j : sources)
    for (auto& d : dep[j])
      if (!(j >= c0 && d.first >= c0)) items.push_back({d.first, j, d.second});
  std::sort(items.begin(), items.end());
  for (size_t a = 0; a < items.size();) {
    size_t b = a;
    while (b < items.size() && items[b][0] == items[a][0]) ++b;
    tasks.push_back({(int)a, (int)b});
    a = b;
  }
}

void build_solve_sched(const Sym& s, bool up, int S, Sched& out) {
  const auto dep = dependents(s, up);
  const auto groups = phase_groups(s, up);
  out = Sched();
  out.S = S;
  out.nphase = (int)groups.size();
  out.ptr.assign(1, 0);
  std::vector<std::array<int, 3>> items;
  std::vector<std::pair<int, int>> tasks;
  std::vector<std::vector<int>> slot_tasks(S);
  std::vector<long long> cost;
  for (int q = 0; q < out.nphase; ++q) {
    phase_tasks(s, dep, groups[q], items, tasks);
    cost.resize(tasks.size());
    for (size_t t = 0; t < tasks.size(); ++t) cost[t] = tasks[t].second - tasks[t].first;
    assign_tasks(cost, S, slot_tasks);
    for (int sl = 0; sl < S; ++sl) {
      for (int t : slot_tasks[sl])
        for (int a = tasks[t].first; a < tasks[t].second; ++a) {
          const int pos = items[a][2];
          out.ent.insert(out.ent.end(), {items[a][0], items[a][1], pos, s.f_tpos[pos]});
        }
      out.ptr.push_back((int)(out.ent.size() / 4));
    }
  }
}

// Pull form of a solve schedule: a row subtracts its terms in few tasks
// rather than one per level of its sources (push), so that a sweep whose
// panel lives in device memory writes each row about once.  Levels count
// from the rows with no sources (level 0, nothing to do); in phase q the
// rows of level <= q are final, and a row of level L finishes in phase L - 1
// (its home phase).  A row with more than kPullCap terms would hold one
// slot for its whole length while the phase's other slots wait, so its terms,
// taken latest source level first, are cut into pieces of kPullCap: the first
// piece in the home phase, each further piece in the phase before the
// previous one when all its sources are final by then (else it joins the
// previous piece).  Pairs inside the chain are left to the chain solve: up,
// the chain rows (last in the order) take their terms from rows before the
// chain in the phases and the chain solve follows; down, the chain is solved
// first, so its rows are final from the start (level 0).
constexpr int kPullCap = 16;

void build_pull_sched(const Sym& s, bool up, int S, Sched& out) {
  const int nx = s.nx, c0 = nx - s.chain_t;
  auto range = [&](int i) -> std::pair<int, int> {
    return up ? std::make_pair(s.f_ptr[i], s.f_diag[i]) : std::make_pair(s.f_diag[i] + 1, s.f_ptr[i + 1]);
  };
  std::vector<int> lev(nx, 0);
  int nlev = 0;
  for (int t = 0; t < nx; ++t) {
    const int i = up ? t : nx - 1 - t;
    int L = 0;
    const auto r = range(i);
    for (int e = r.first; e < r.second; ++e) {
      const int j = s.f_col[e];
      if (i >= c0 && j >= c0) continue;
      L = std::max(L, lev[j] + 1);
    }
    lev[i] = L;
    nlev = std::max(nlev, L);
  }
  // pieces (row, entry positions) per phase
  std::vector<std::vector<std::pair<int, std::vector<int>>>> ph(nlev);
  std::vector<int> es;
  for (int i = 0; i < nx; ++i) {
    es.clear();
    const auto r = range(i);
    for (int e = r.first; e < r.second; ++e)
      if (!(i >= c0 && s.f_col[e] >= c0)) es.push_back(e);
    if (es.empty()) continue;
    std::stable_sort(es.begin(), es.end(), [&](int x, int y) { return lev[s.f_col[x]] > lev[s.f_col[y]]; });
    std::vector<std::pair<int, std::vector<int>>> pieces;
    for (size_t k = 0; k < es.size(); k += kPullCap) {
      std::vector<int> ch(es.begin() + k, es.begin() + std::min(es.size(), k + kPullCap));
      const int ml = lev[s.f_col[ch[0]]];  // the piece's latest source level
      if (pieces.empty()) pieces.push_back({lev[i] - 1, ch});
      else if (pieces.back().first - 1 >= ml) pieces.push_back({pieces.back().first - 1, ch});
      else pieces.back().second.insert(pieces.back().second.end(), ch.begin(), ch.end());
    }
    for (auto& pc : pieces) {
      std::sort(pc.second.begin(), pc.second.end());  // terms in pattern order
      ph[pc.first].push_back({i, std::move(pc.second)});
    }
  }
  out = Sched();
  out.S = S;
  out.nphase = nlev;
  out.ptr.assign(1, 0);
  std::vector<std::vector<int>> slot_tasks(S);
  std::vector<long long> cost;
  for (int q = 0; q < nlev; ++q) {
    const auto& tq = ph[q];
    cost.resize(tq.size());
    for (size_t t = 0; t < tq.size(); ++t) cost[t] = (long long)tq[t].second.size();
    assign_tasks(cost, S, slot_tasks);
    for (int sl = 0; sl < S; ++sl) {
      for (int t : slot_tasks[sl]) {
        const int i = tq[t].first;
        for (int e : tq[t].second) out.ent.insert(out.ent.end(), {i, s.f_col[e], e, s.f_tpos[e]});
      }
      out.ptr.push_back((int)(out.ent.size() / 4));
    }
  }
}

// Refactorisation items: the entry l_ik of row i, taken when row k (level q)
// is final, costs one multiply by 1/u_kk and one update of row i per entry of
// the U part of row k.  upd receives, per item, the positions of (i, j) for
// the U columns j of row k in order.  Items inside the chain are left to the
// chain factorisation.
std::string build_fac_sched(const Sym& s, int S, Sched& out, std::vector<int>& upd) {
  const auto dep = dependents(s, true);
  const auto groups = phase_groups(s, true);
  out = Sched();
  out.S = S;
  out.nphase = (int)groups.size();
  out.ptr.assign(1, 0);
  upd.clear();
  std::vector<std::array<int, 3>> items;
  std::vector<std::pair<int, int>> tasks;
  std::vector<std::vector<int>> slot_tasks(S);
  std::vector<long long> cost;
  for (int q = 0; q < out.nphase; ++q) {
    phase_tasks(s, dep, groups[q], items, tasks);
    cost.assign(tasks.size(), 0);
    for (size_t t = 0; t < tasks.size(); ++t)
      for (int a = tasks[t].first; a < tasks[t].second; ++a) {
        const int k = items[a][1];
        cost[t] += 1 + (s.f_ptr[k + 1] - s.f_diag[k] - 1);
      }
    assign_tasks(cost, S, slot_tasks);
    for (int sl = 0; sl < S; ++sl) {
      for (int t : slot_tasks[sl])
        for (int a = tasks[t].first; a < tasks[t].second; ++a) {
          const int i = items[a][0], k = items[a][1], pos = items[a][2];
          const int ulen = s.f_ptr[k + 1] - s.f_diag[k] - 1;
          out.ent.insert(out.ent.end(), {pos, s.f_diag[k], ulen, (int)upd.size()});
          for (int e = s.f_diag[k] + 1; e < s.f_ptr[k + 1]; ++e) {
            const int tgt = find_pos(s.f_ptr, s.f_col, i, s.f_col[e]);
            if (tgt < 0) return "internal: filled pattern not closed under elimination";
            upd.push_back(tgt);
          }
        }
      out.ptr.push_back((int)(out.ent.size() / 4));
    }
  }
  return "";
}

// The chain: a suffix of the elimination order (at most kChainMax rows) that
// the solves and the refactorisation take sequentially in registers.  No row
// before it depends on it in the up direction and it depends on nothing
// before it in the down direction, so any suffix is valid; its length is the
// one with the fewest barrier-separated phases, counting a chain step as an
// eighth of a phase.  chain_pos[a t + b] is the position of (c0 + a, c0 + b)
// in the filled pattern, -1 where structurally zero.
void find_chain(Sym& s, int chain_req) {
  const int nx = s.nx;
  int best_t = 0;
  double best = 1e300;
  const int tmax = chain_req > 0 ? chain_req : chain_req < 0 ? 0 : kChainMax;
  for (int t = 0; t <= tmax && t <= nx; ++t) {
    const double cost = (double)phase_groups_t(s, true, t).size() + (double)phase_groups_t(s, false, t).size() +
                        t / 8.0;
    if (cost < best - 1e-9) { best = cost; best_t = t; }
  }
  const int t = best_t < 2 ? 0 : best_t;
  s.chain_t = t;
  s.chain_pos.assign((size_t)t * t, -1);
  const int c0 = nx - t;
  for (int a = 0; a < t; ++a)
    for (int b = 0; b < t; ++b) s.chain_pos[a * t + b] = find_pos(s.f_ptr, s.f_col, c0 + a, c0 + b);
}
}  // namespace

LdsSizes lds_sizes(const Sym& s, int w, int variant, int spw) {
  LdsSizes z;
  z.nx = s.nx; z.nu = s.nu; z.nz = s.nz;
  z.nnz_f = (int)s.f_col.size(); z.nnz_k = (int)s.k_col.size(); z.nnz_gu = (int)s.gu_col.size();
  z.nnz_l = s.nnz_l;
  z.nlu = (int)s.lvu_ptr.size() - 1;
  z.nph_u = std::max(0, z.nlu - 1);
  z.nph_d = std::max(0, (int)s.lvd_ptr.size() - 1);  // the chain's merged phase may add one
  z.nph_ru = z.nph_u;  // the reduction runs in LDS with push schedules only
  z.nph_rd = z.nph_d;
  z.n_upd = (int)(s.lu_flops - s.nnz_l);
  z.w = w; z.variant = variant; z.spw = spw;
  z.upd_lds = s.upd_lds ? 1 : 0;
  z.nnz_h = (int)s.h_col.size(); z.m = s.m;
  z.chain_t = s.chain_t;
  return z;
}

std::string build_symbolic(const rkkt_network& net, int N, const rkkt_options* opt, Sym& s) {
  const int col_tile_req = opt ? opt->col_tile : 0, variant_req = opt ? opt->variant : 0;
  const int spw_req = opt ? opt->scen_per_group : 0, chain_req = opt ? opt->chain_rows : 0;
  if (spw_req != 0 && spw_req != 1 && spw_req != 2 && spw_req != 4) return "scen_per_group must be 0, 1, 2 or 4";
  if (chain_req < -1 || chain_req > kChainMax) return "chain_rows must be in [-1, 32]";
  const int form_req = opt ? opt->sweep_form : 0;
  if (form_req < 0 || form_req > 2) return "sweep_form must be 0, 1 or 2";
  char msg[256];
  const int nb = net.n_bus, nl = net.n_line, ng = net.n_gen, nload = net.n_load;
  if (nb < 2 || nl < 1 || ng < 1 || nload < 0 || N < 1) return "bad sizes";
  if (!net.line_from || !net.line_to || !net.r || !net.x || !net.b || !net.rate ||
      !net.gen_bus || !net.pmin || !net.pmax || !net.qmin || !net.qmax || !net.c2 ||
      !net.c1 || !net.c0 || !net.vmin || !net.vmax || (nload > 0 && !net.load_bus))
    return "null network array";
  for (int l = 0; l < nl; ++l) {
    int f = net.line_from[l], t = net.line_to[l];
    if (f < 0 || f >= nb || t < 0 || t >= nb || f == t) {
      snprintf(msg, sizeof msg, "line %d has bad end buses (%d, %d)", l, f, t);
      return msg;
    }
  }
  std::vector<int> gen_of_bus(nb, -1);
  for (int g = 0; g < ng; ++g) {
    int b = net.gen_bus[g];
    if (b < 0 || b >= nb) return "generator bus out of range";
    if (gen_of_bus[b] >= 0) return "two generators on one bus";
    gen_of_bus[b] = g;
  }
  if (net.ref_bus < 0 || net.ref_bus >= nb || gen_of_bus[net.ref_bus] < 0)
    return "ref_bus must be a generator bus";
  {
    std::vector<char> seen(nb, 0);
    for (int i = 0; i < nload; ++i) {
      int b = net.load_bus[i];
      if (b < 0 || b >= nb) return "load bus out of range";
      if (seen[b]) return "two loads on one bus";
      seen[b] = 1;
    }
  }
  s = Sym();
  s.nb = nb; s.nl = nl; s.ng = ng; s.nload = nload; s.N = N;
  s.ref = net.ref_bus;
  s.gref = gen_of_bus[s.ref];
  s.nx = 2 * nb - ng - 1;
  s.nu = 2 * ng - 1;
  s.m = 2 * nl + ng + 1;
  s.nz = s.nx + s.nu;
  const int nx = s.nx, nu = s.nu;
  s.gen_bus.assign(net.gen_bus, net.gen_bus + ng);
  for (int g = 0; g < ng; ++g)
    if (g != s.gref) s.gnr.push_back(g);

  // external variable maps (the order of the public interface)
  s.th_src.assign(nb, -1);
  s.v_src.assign(nb, 0);
  s.prow.assign(nb, -1);
  s.qrow.assign(nb, 0);
  s.pg_u.assign(nb, -1);
  {
    int k = 0;
    for (int b = 0; b < nb; ++b)
      if (b != s.ref) { s.th_src[b] = k; s.prow[b] = k; ++k; }
    for (int b = 0; b < nb; ++b)
      if (gen_of_bus[b] < 0) { s.v_src[b] = k; s.qrow[b] = k; ++k; }
      else { s.v_src[b] = -(1 + gen_of_bus[b]); s.qrow[b] = -(1 + gen_of_bus[b]); }
    if (k != nx) return "internal: x size";
    for (size_t j = 0; j < s.gnr.size(); ++j) s.pg_u[s.gen_bus[s.gnr[j]]] = ng + (int)j;
  }
  s.line_f.assign(net.line_from, net.line_from + nl);
  s.line_t.assign(net.line_to, net.line_to + nl);
  std::vector<std::vector<std::pair<int, int>>> ends(nb);  // (line, end)
  for (int l = 0; l < nl; ++l) {
    ends[s.line_f[l]].push_back({l, 0});
    ends[s.line_t[l]].push_back({l, 1});
  }

  // ---- fill-reducing ordering of G_x (pattern of G_x + G_x^T, external order)
  auto ext_var = [&](int b, int which) -> int {  // which 0: theta, 1: v ; -1 if not an x var
    if (which == 0) return s.th_src[b];
    return s.v_src[b] >= 0 ? s.v_src[b] : -1;
  };
  {
    std::vector<std::vector<int>> adj(nx);
    auto add_row = [&](int r, int b) {
      for (auto& le : ends[b]) {
        int l = le.first;
        int bb[2] = {s.line_f[l], s.line_t[l]};
        for (int q = 0; q < 2; ++q)
          for (int w = 0; w < 2; ++w) {
            int c = ext_var(bb[q], w);
            if (c >= 0 && c != r) { adj[r].push_back(c); adj[c].push_back(r); }
          }
      }
    };
    for (int b = 0; b < nb; ++b) {
      if (s.prow[b] >= 0) add_row(s.prow[b], b);
      if (s.qrow[b] >= 0) add_row(s.qrow[b], b);
    }
    for (auto& a : adj) {
      std::sort(a.begin(), a.end());
      a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    std::vector<std::vector<int>> fill;
    std::vector<int> order = minimum_degree(nx, adj, fill);
    s.perm = order;
    s.pinv.assign(nx, 0);
    for (int i = 0; i < nx; ++i) s.pinv[order[i]] = i;
    // filled pattern in internal order: row i has U part = pinv(fill[perm[i]])
    std::vector<std::vector<int>> up(nx), lo(nx);
    for (int i = 0; i < nx; ++i) {
      for (int w : fill[order[i]]) up[i].push_back(s.pinv[w]);
      std::sort(up[i].begin(), up[i].end());
      for (int j : up[i]) {
        if (j <= i) return "internal: fill order";
        lo[j].push_back(i);
      }
    }
    s.f_ptr.assign(nx + 1, 0);
    for (int i = 0; i < nx; ++i) s.f_ptr[i + 1] = s.f_ptr[i] + (int)(lo[i].size() + 1 + up[i].size());
    s.f_col.resize(s.f_ptr[nx]);
    s.f_diag.resize(nx);
    for (int i = 0; i < nx; ++i) {
      int p = s.f_ptr[i];
      for (int k : lo[i]) s.f_col[p++] = k;  // lo[i] is ascending by construction
      s.f_diag[i] = p;
      s.f_col[p++] = i;
      for (int j : up[i]) s.f_col[p++] = j;
    }
    s.f_tpos.resize(s.f_col.size());
    for (int i = 0; i < nx; ++i)
      for (int e = s.f_ptr[i]; e < s.f_ptr[i + 1]; ++e) {
        int t = find_pos(s.f_ptr, s.f_col, s.f_col[e], i);
        if (t < 0) return "internal: filled pattern not symmetric";
        s.f_tpos[e] = t;
      }
    s.lu_flops = 0;
    for (int i = 0; i < nx; ++i)
      for (int e = s.f_ptr[i]; e < s.f_diag[i]; ++e) {
        int k = s.f_col[e];
        s.lu_flops += 1 + (s.f_ptr[k + 1] - s.f_diag[k] - 1);
      }
    // level schedules
    std::vector<int> lvl(nx, 0);
    int nlu = 0;
    for (int i = 0; i < nx; ++i) {
      int L = 0;
      for (int e = s.f_ptr[i]; e < s.f_diag[i]; ++e) L = std::max(L, lvl[s.f_col[e]] + 1);
      lvl[i] = L;
      nlu = std::max(nlu, L + 1);
    }
    s.lvu_ptr.assign(nlu + 1, 0);
    for (int i = 0; i < nx; ++i) s.lvu_ptr[lvl[i] + 1]++;
    for (int q = 0; q < nlu; ++q) s.lvu_ptr[q + 1] += s.lvu_ptr[q];
    s.lvu_rows.resize(nx);
    {
      std::vector<int> cur(s.lvu_ptr.begin(), s.lvu_ptr.end() - 1);
      for (int i = 0; i < nx; ++i) s.lvu_rows[cur[lvl[i]]++] = i;
    }
    int nld = 0;
    for (int i = nx - 1; i >= 0; --i) {
      int L = 0;
      for (int e = s.f_diag[i] + 1; e < s.f_ptr[i + 1]; ++e) L = std::max(L, lvl[s.f_col[e]] + 1);
      lvl[i] = L;
      nld = std::max(nld, L + 1);
    }
    s.lvd_ptr.assign(nld + 1, 0);
    for (int i = 0; i < nx; ++i) s.lvd_ptr[lvl[i] + 1]++;
    for (int q = 0; q < nld; ++q) s.lvd_ptr[q + 1] += s.lvd_ptr[q];
    s.lvd_rows.resize(nx);
    {
      std::vector<int> cur(s.lvd_ptr.begin(), s.lvd_ptr.end() - 1);
      for (int i = 0; i < nx; ++i) s.lvd_rows[cur[lvl[i]]++] = i;
    }
  }

  s.nnz_l = 0;
  for (int i = 0; i < nx; ++i) s.nnz_l += s.f_diag[i] - s.f_ptr[i];

  // ---- internal z index of the locals of every line
  auto zvar = [&](int b, int which) -> int {
    if (which == 0) return s.th_src[b] >= 0 ? s.pinv[s.th_src[b]] : -1;
    return s.v_src[b] >= 0 ? s.pinv[s.v_src[b]] : nx + (-s.v_src[b] - 1);
  };
  s.line_loc.resize(4 * nl);
  for (int l = 0; l < nl; ++l) {
    s.line_loc[4 * l + 0] = zvar(s.line_f[l], 0);
    s.line_loc[4 * l + 1] = zvar(s.line_t[l], 0);
    s.line_loc[4 * l + 2] = zvar(s.line_f[l], 1);
    s.line_loc[4 * l + 3] = zvar(s.line_t[l], 1);
  }

  // ---- Jacobian rows: gradient of a bus injection (P: type 0, Q: type 1)
  auto bus_row = [&](int b, int type, SparseRow& row) {
    for (auto& le : ends[b]) {
      int l = le.first, e = le.second;
      for (int q = 0; q < 4; ++q) {
        int v = s.line_loc[4 * l + q];
        if (v < 0) continue;
        row[v].src.push_back(l * kLVsize + 14 * e + (type == 0 ? kLVdP : kLVdQ) + q);
      }
    }
  };
  std::vector<SparseRow> grow(nx);  // by internal row
  for (int b = 0; b < nb; ++b) {
    if (s.prow[b] >= 0) {
      SparseRow& row = grow[s.pinv[s.prow[b]]];
      bus_row(b, 0, row);
      if (s.pg_u[b] >= 0) row[nx + s.pg_u[b]].c = -1.0;
    }
    if (s.qrow[b] >= 0) bus_row(b, 1, grow[s.pinv[s.qrow[b]]]);
  }
  std::vector<SparseRow> hrow(s.m);
  bus_row(s.ref, 0, hrow[0]);
  for (int g = 0; g < ng; ++g) bus_row(s.gen_bus[g], 1, hrow[1 + g]);
  for (int l = 0; l < nl; ++l)
    for (int e = 0; e < 2; ++e) {
      SparseRow& row = hrow[1 + ng + e * nl + l];
      for (int q = 0; q < 4; ++q) {
        int v = s.line_loc[4 * l + q];
        if (v >= 0) row[v].src.push_back(l * kLVsize + 14 * e + kLVdS + q);
      }
    }

  // ---- EV gather lists
  s.off_P = 0;
  s.off_Q = nb;
  s.ev_ptr.assign(1, 0);
  auto push_ev = [&](const std::vector<int>& src, double c) {
    s.ev_src.insert(s.ev_src.end(), src.begin(), src.end());
    s.ev_ptr.push_back((int)s.ev_src.size());
    s.ev_const.push_back(c);
  };
  for (int type = 0; type < 2; ++type)
    for (int b = 0; b < nb; ++b) {
      std::vector<int> src;
      for (auto& le : ends[b]) src.push_back(le.first * kLVsize + 14 * le.second + (type == 0 ? kLVP : kLVQ));
      push_ev(src, 0.0);
    }
  s.off_gx = (int)s.ev_const.size();
  s.gx_ptr.assign(nx + 1, 0);
  for (int i = 0; i < nx; ++i) {
    for (auto& kv : grow[i])
      if (kv.first < nx) { s.gx_col.push_back(kv.first); push_ev(kv.second.src, kv.second.c); }
    s.gx_ptr[i + 1] = (int)s.gx_col.size();
  }
  s.off_gu = (int)s.ev_const.size();
  s.gu_ptr.assign(nx + 1, 0);
  for (int i = 0; i < nx; ++i) {
    for (auto& kv : grow[i])
      if (kv.first >= nx) { s.gu_col.push_back(kv.first - nx); push_ev(kv.second.src, kv.second.c); }
    s.gu_ptr[i + 1] = (int)s.gu_col.size();
  }
  s.off_h = (int)s.ev_const.size();
  s.h_ptr.assign(s.m + 1, 0);
  for (int r = 0; r < s.m; ++r) {
    for (auto& kv : hrow[r]) { s.h_col.push_back(kv.first); push_ev(kv.second.src, kv.second.c); }
    s.h_ptr[r + 1] = (int)s.h_col.size();
  }
  s.n_ev = (int)s.ev_const.size();
  for (int i = 0; i < nx; ++i)
    if (s.gx_ptr[i + 1] == s.gx_ptr[i] || find_pos(s.gx_ptr, s.gx_col, i, i) < 0)
      return "G_x has a structurally zero diagonal (isolated bus?)";

  // G_x by column
  s.gxc_ptr.assign(nx + 1, 0);
  for (int c : s.gx_col) s.gxc_ptr[c + 1]++;
  for (int c = 0; c < nx; ++c) s.gxc_ptr[c + 1] += s.gxc_ptr[c];
  s.gxc_row.resize(s.gx_col.size());
  s.gxc_pos.resize(s.gx_col.size());
  {
    std::vector<int> cur(s.gxc_ptr.begin(), s.gxc_ptr.end() - 1);
    for (int i = 0; i < nx; ++i)
      for (int e = s.gx_ptr[i]; e < s.gx_ptr[i + 1]; ++e) {
        int c = s.gx_col[e];
        s.gxc_row[cur[c]] = i;
        s.gxc_pos[cur[c]] = e;
        cur[c]++;
      }
  }
  // G_u by column
  s.guc_ptr.assign(nu + 1, 0);
  for (int c : s.gu_col) s.guc_ptr[c + 1]++;
  for (int c = 0; c < nu; ++c) s.guc_ptr[c + 1] += s.guc_ptr[c];
  s.guc_row.resize(s.gu_col.size());
  s.guc_pos.resize(s.gu_col.size());
  {
    std::vector<int> cur(s.guc_ptr.begin(), s.guc_ptr.end() - 1);
    for (int i = 0; i < nx; ++i)
      for (int e = s.gu_ptr[i]; e < s.gu_ptr[i + 1]; ++e) {
        int c = s.gu_col[e];
        s.guc_row[cur[c]] = i;
        s.guc_pos[cur[c]] = e;
        cur[c]++;
      }
  }
  // H transposed
  s.ht_ptr.assign(s.nz + 1, 0);
  for (int v : s.h_col) s.ht_ptr[v + 1]++;
  for (int v = 0; v < s.nz; ++v) s.ht_ptr[v + 1] += s.ht_ptr[v];
  s.ht_row.resize(s.h_col.size());
  s.ht_pos.resize(s.h_col.size());
  {
    std::vector<int> cur(s.ht_ptr.begin(), s.ht_ptr.end() - 1);
    for (int r = 0; r < s.m; ++r)
      for (int e = s.h_ptr[r]; e < s.h_ptr[r + 1]; ++e) {
        int v = s.h_col[e];
        s.ht_row[cur[v]] = r;
        s.ht_pos[cur[v]] = e;
        cur[v]++;
      }
  }
  s.h0pos.assign(s.nz, -1);
  for (int e = s.h_ptr[0]; e < s.h_ptr[1]; ++e) s.h0pos[s.h_col[e]] = e;

  // ---- K = W + H^T Sigma_s H (+ diagonals): pattern and gather lists
  std::map<std::pair<int, int>, KEntry> K;
  for (int l = 0; l < nl; ++l)
    for (int a = 0; a < 4; ++a)
      for (int b = a; b < 4; ++b) {
        int va = s.line_loc[4 * l + a], vb = s.line_loc[4 * l + b];
        if (va < 0 || vb < 0) continue;
        int src = l * kLHsize + lh_index(a, b);
        K[{va, vb}].wsrc.push_back(src);
        if (va != vb) K[{vb, va}].wsrc.push_back(src);
      }
  const double aref = 1e4 * net.c2[s.gref];
  for (int e1 = s.h_ptr[0]; e1 < s.h_ptr[1]; ++e1)
    for (int e2 = s.h_ptr[0]; e2 < s.h_ptr[1]; ++e2) {
      KEntry& ke = K[{s.h_col[e1], s.h_col[e2]}];
      ke.wprod.push_back({e1, e2});
      ke.wcoef.push_back(2.0 * aref);
    }
  for (size_t j = 0; j < s.gnr.size(); ++j) {
    int v = nx + ng + (int)j;
    K[{v, v}].wconst += 2.0 * 1e4 * net.c2[s.gnr[j]];
  }
  for (int r = 0; r < s.m; ++r)
    for (int e1 = s.h_ptr[r]; e1 < s.h_ptr[r + 1]; ++e1)
      for (int e2 = s.h_ptr[r]; e2 < s.h_ptr[r + 1]; ++e2)
        K[{s.h_col[e1], s.h_col[e2]}].trip.push_back({r, e1, e2});
  for (int v = 0; v < s.nz; ++v) K[{v, v}];
  s.k_ptr.assign(s.nz + 1, 0);
  s.w_ptr.assign(1, 0);
  s.wp_ptr.assign(1, 0);
  s.t_ptr.assign(1, 0);
  for (auto& kv : K) {
    int r = kv.first.first, c = kv.first.second;
    s.k_ptr[r + 1]++;
    s.k_col.push_back(c);
    const KEntry& ke = kv.second;
    s.w_src.insert(s.w_src.end(), ke.wsrc.begin(), ke.wsrc.end());
    s.w_ptr.push_back((int)s.w_src.size());
    for (size_t q = 0; q < ke.wprod.size(); ++q) {
      s.wp_a.push_back(ke.wprod[q][0]);
      s.wp_b.push_back(ke.wprod[q][1]);
      s.wp_coef.push_back(ke.wcoef[q]);
    }
    s.wp_ptr.push_back((int)s.wp_a.size());
    s.w_const.push_back(ke.wconst);
    for (auto& t : ke.trip) {
      s.t_row.push_back(t[0]);
      s.t_a.push_back(t[1]);
      s.t_b.push_back(t[2]);
    }
    s.t_ptr.push_back((int)s.t_row.size());
  }
  for (int r = 0; r < s.nz; ++r) s.k_ptr[r + 1] += s.k_ptr[r];
  s.k_diag.resize(s.nz);
  s.k_usplit.resize(s.nz);
  for (int r = 0; r < s.nz; ++r) {
    s.k_diag[r] = find_pos(s.k_ptr, s.k_col, r, r);
    auto b = s.k_col.begin() + s.k_ptr[r], e = s.k_col.begin() + s.k_ptr[r + 1];
    s.k_usplit[r] = (int)(std::lower_bound(b, e, nx) - s.k_col.begin());
  }
  // K-row items of the product K Z in the LDS-mode reduction: one per row
  // (its x-part entries as one run), longest first, so that the threads
  // holding the longest rows start them first and the shortest rows are the
  // second items; none when they need more than kKzItems items of four per
  // thread.  (Cutting the long rows into shorter runs, summed in order one
  // round each, measured no faster on the 118-bus grid.)
  if (4LL * s.nz <= (long long)kKzItems * kRedThreads) {
    std::vector<std::array<int, 4>> pc;
    for (int r = 0; r < s.nz; ++r) pc.push_back({r, s.k_ptr[r], s.k_usplit[r], 0});
    std::stable_sort(pc.begin(), pc.end(), [](const std::array<int, 4>& a, const std::array<int, 4>& b) {
      return a[2] - a[1] > b[2] - b[1];
    });
    for (auto& t : pc) s.kz_items.insert(s.kz_items.end(), t.begin(), t.end());
    s.kz_rounds = 1;
  }

  // G_x entries inside the filled pattern
  s.gx2f.resize(s.gx_col.size());
  for (int i = 0; i < nx; ++i)
    for (int e = s.gx_ptr[i]; e < s.gx_ptr[i + 1]; ++e) {
      int p = find_pos(s.f_ptr, s.f_col, i, s.gx_col[e]);
      if (p < 0) return "internal: G_x entry outside the filled pattern";
      s.gx2f[e] = p;
    }

  // boxes
  {
    const double inf = std::numeric_limits<double>::infinity();
    s.xl.assign(nx, -inf);
    s.xu.assign(nx, inf);
    for (int b = 0; b < nb; ++b)
      if (s.v_src[b] >= 0) { s.xl[s.v_src[b]] = net.vmin[b]; s.xu[s.v_src[b]] = net.vmax[b]; }
    s.ul.assign(nu, 0.0);
    s.uu.assign(nu, 0.0);
    for (int g = 0; g < ng; ++g) { s.ul[g] = net.vmin[s.gen_bus[g]]; s.uu[g] = net.vmax[s.gen_bus[g]]; }
    for (size_t j = 0; j < s.gnr.size(); ++j) {
      s.ul[ng + j] = net.pmin[s.gnr[j]];
      s.uu[ng + j] = net.pmax[s.gnr[j]];
    }
    s.sl.assign(s.m, -inf);
    s.su.assign(s.m, inf);
    s.sl[0] = -net.pmax[s.gref];
    s.su[0] = -net.pmin[s.gref];
    for (int g = 0; g < ng; ++g) { s.sl[1 + g] = -net.qmax[g]; s.su[1 + g] = -net.qmin[g]; }
    for (int l = 0; l < nl; ++l) {
      s.sl[1 + ng + l] = -net.rate[l] * net.rate[l];
      s.sl[1 + ng + nl + l] = -net.rate[l] * net.rate[l];
    }
  }

  find_chain(s, chain_req);  // depends on the level structure only

  // ---- launch shapes.  Packed 16-bit schedule entries need every index
  // below 2^16, which holds whenever the data they index fits in LDS.
  const long long lds_max = 160 * 1024;
  const bool pack_ok = nx < 65536 && s.f_col.size() < 65536 && s.lu_flops < 65536;
  // refactorisation and step: up to 4 scenarios per workgroup, one
  // wavefront each, when a scenario's LU values and vectors fit in LDS; the
  // automatic choice stops at 2 (at 118 buses and 128 scenarios the pass
  // measured 232 us with 2 or 1 scenarios per workgroup against 234 us with 4)
  s.spw = 0;
  for (int spw : {4, 2, 1}) {
    if (spw_req > 0 ? spw > spw_req : spw > 2) continue;
    for (int staged : {1, 0}) {
      s.upd_lds = staged;
      if (pack_ok && refactor_lds_bytes(lds_sizes(s, 1, 1, spw)) <= lds_max) {
        s.spw = spw;
        break;
      }
    }
    if (s.spw) break;
  }
  s.lds_group = s.spw > 0;
  if (!s.lds_group) s.spw = 1;
  s.group = s.lds_group ? kGroupLds : kRedThreads;
  s.lds_step = pack_ok && step_lds_bytes(lds_sizes(s, 1, 1, 1)) <= lds_max;
  s.step_group = s.lds_step ? kGroupLds : kRedThreads;
  // reduction: the fewest column tiles whose workgroup fits in LDS, else
  // panels of 64 columns in global memory
  if (variant_req < 0 || variant_req > 2) return "variant must be 0, 1 or 2";
  if (col_tile_req < 0 || col_tile_req > 64) return "col_tile must be in [0, 64]";
  auto fits = [&](int w, int v) { return pack_ok && reduce_lds_bytes(lds_sizes(s, w, v, 1)) <= lds_max; };
  auto pick_tile = [&](int v) {
    if (nu > 32 && fits(64, v)) return 64;  // one slot per wavefront
    for (int tiles = 1; tiles <= 64 && tiles <= nu; ++tiles) {
      const int w = (nu + tiles - 1) / tiles;
      if (w <= 64 && fits(w, v)) return w;
    }
    return 0;
  };
  if (variant_req == 0) s.variant = pick_tile(2) > 0 ? 2 : 1;  // stacked product when it stays on chip
  else s.variant = variant_req;
  if (col_tile_req > 0) s.col_tile = std::min(col_tile_req, nu);
  else {
    s.col_tile = pick_tile(s.variant);
    if (s.col_tile == 0) s.col_tile = std::min(64, nu);
  }
  s.lds_reduce = form_req != 2 && fits(s.col_tile, s.variant);
  s.sweep_form = form_req != 0 ? form_req : s.lds_reduce ? 1 : 2;
  s.lds_resident = s.lds_reduce && s.lds_group && s.lds_step;
  // stacked panels of the product variant: rows (x rows then u rows) of every
  // scenario, columns padded to a multiple of 64 (the reduction's widest tile)
  s.nu_pad = (nu + 63) / 64 * 64;
  {
    // row chunks of the stacked product: about 256 workgroups over the
    // super-tiles of 7 x 7 16-column blocks, at least 64 rows per chunk
    const long long rows = (long long)N * s.nz;
    const long long T = ((nu + 15) / 16 + 6) / 7;
    const long long tiles = T * (T + 1) / 2;
    long long nc = std::max(1LL, 256 / tiles);
    nc = std::min(nc, std::max(1LL, rows / 64));
    // chunks of whole slabs; no chunk starts past the last row
    const long long per = ((rows + nc - 1) / nc + kSpSlab - 1) / kSpSlab * kSpSlab;
    nc = (rows + per - 1) / per;
    s.nchunk = (int)nc;
  }
  // schedules
  if (s.sweep_form == 2) {
    build_pull_sched(s, true, kRedThreads / s.col_tile, s.red_up);
    build_pull_sched(s, false, kRedThreads / s.col_tile, s.red_dn);
  } else {
    build_solve_sched(s, true, kRedThreads / s.col_tile, s.red_up);
    build_solve_sched(s, false, kRedThreads / s.col_tile, s.red_dn);
  }
  build_solve_sched(s, true, s.step_group, s.stp_up);
  build_solve_sched(s, false, s.step_group, s.stp_dn);
  {
    std::string m = build_fac_sched(s, s.group, s.fac, s.upd_dst);
    if (!m.empty()) return m;
  }
  // every schedule holds the pairs outside the chain exactly once (the
  // kernels size their LDS images from one count)
  for (const Sched* sc : {&s.red_dn, &s.stp_up, &s.stp_dn, &s.fac})
    if (sc->ent.size() != s.red_up.ent.size()) return "internal: schedule sizes differ";
  return "";
}

}  // namespace rkkt

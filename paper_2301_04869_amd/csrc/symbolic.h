// Host-side symbolic analysis of the block AC-OPF reduced-KKT path.
//
// Everything here depends only on the network (never on values), is computed
// once per problem and shared by all scenario blocks: the paper's blocks share
// one sparsity pattern (parallel AD section: Jacobians of the blocks share
// their pattern; parallel KKT section: batched LU on a shared pattern).
#pragma once

#include <string>
#include <vector>

#include "layout.h"
#include "rkkt.h"

namespace rkkt {

// Level-sliced schedule of a triangular sweep over S slots.  Phase q starts
// once the rows of level q are final; every task of the phase is one
// dependent row together with its entries whose source row lies in level q,
// and a slot runs its tasks of the phase one after another.  The entries of
// (phase q, slot t) are ent[4 ptr[q S + t] .. 4 ptr[q S + t + 1]); solve
// entries are (dest row, source row, position of (dest, source) in the filled
// pattern, position of (source, dest)); refactorisation entries are (position
// of l_ik, position of u_kk, length of the U part of row k, first update
// target in upd_dst).
struct Sched {
  int S = 0, nphase = 0;
  std::vector<int> ptr, ent;
};

struct Sym {
  int nb = 0, nl = 0, ng = 0, nload = 0, ref = 0, gref = 0;
  int nx = 0, nu = 0, m = 0, nz = 0, N = 0;
  int col_tile = 0;
  bool lds_resident = true;  // every level-scheduled kernel keeps its data in LDS
  bool lds_reduce = true;    // the reduction's panels and factors sit in LDS
  int sweep_form = 1;        // reduction schedules: 1 push (per source level), 2 pull (per destination row)
  bool lds_group = true;     // the refactorisation keeps its scenarios in LDS
  bool lds_step = true;      // the step keeps its scenario in LDS

  // internal x order: xhat = perm applied to the external order
  std::vector<int> perm;  // perm[ihat] = i_ext
  std::vector<int> pinv;  // pinv[i_ext] = ihat

  // buses
  std::vector<int> th_src;   // external x index of theta_b, -1 for the reference bus
  std::vector<int> v_src;    // external x index of V_b (PQ), or -(1+u index) (generator bus)
  std::vector<int> prow;     // external g row of the P balance of b, -1 for ref
  std::vector<int> qrow;     // external g row of the Q balance of b (PQ) or -(1+gen) (gen bus)
  std::vector<int> pg_u;     // u index of Pg at bus b (non-ref generator bus) or -1
  std::vector<int> gnr;      // non-reference generators, generator order
  // boxes (+-inf when absent): x (external order), u, s = -h
  std::vector<double> xl, xu, ul, uu, sl, su;
  std::vector<int> gen_bus;

  // lines: internal z index of the locals (th_f, th_t, v_f, v_t), -1 = constant
  std::vector<int> line_f, line_t, line_loc;

  // evaluation outputs EV = [P_b (nb) | Q_b (nb) | Gx values | Gu values | H values]
  int n_ev = 0, off_P = 0, off_Q = 0, off_gx = 0, off_gu = 0, off_h = 0;
  std::vector<int> ev_ptr, ev_src;
  std::vector<double> ev_const;

  // G_x (internal rows and columns), CSR; value k is EV[off_gx + k]
  std::vector<int> gx_ptr, gx_col;
  // G_x by column: internal row and value index
  std::vector<int> gxc_ptr, gxc_row, gxc_pos;
  // G_u (internal rows), CSR; value k is EV[off_gu + k]
  std::vector<int> gu_ptr, gu_col;
  // G_u by column: internal row and value index
  std::vector<int> guc_ptr, guc_row, guc_pos;
  // H (external rows), CSR with internal z columns; value k is EV[off_h + k]
  std::vector<int> h_ptr, h_col;
  // H transposed: for internal z var, (row, value index)
  std::vector<int> ht_ptr, ht_row, ht_pos;
  // position of every z var in H row 0 (gradient of the reference output), -1 if none
  std::vector<int> h0pos;

  // K over internal z = (xhat, u): CSR, full symmetric storage, sorted columns
  std::vector<int> k_ptr, k_col, k_diag, k_usplit;  // k_usplit[r]: first entry with col >= nx
  // pieces of the K rows for the product K Z in the LDS-mode reduction, as
  // (row, first entry, end entry of its x part, index of the piece within
  // its row), longest first; kz_rounds = most pieces of one row (empty when
  // they need more than kKzItems items of four per thread)
  std::vector<int> kz_items;
  int kz_rounds = 0;
  // W gather: LH sources, product terms (coef * Hval[a] * Hval[b]), constant (times obj weight)
  std::vector<int> w_ptr, w_src;
  std::vector<int> wp_ptr, wp_a, wp_b;
  std::vector<double> wp_coef, w_const;
  // condensation triplets: K[e] += sigma_s[row] * Hval[a] * Hval[b]
  std::vector<int> t_ptr, t_row, t_a, t_b;

  // filled LU pattern of P G_x P^T (internal order), CSR with sorted columns
  std::vector<int> f_ptr, f_col, f_diag, f_tpos;
  std::vector<int> gx2f;                       // F position of every G_x entry
  std::vector<int> lvu_ptr, lvu_rows, lvd_ptr, lvd_rows;
  long long lu_flops = 0;

  int nnz_l = 0;  // strictly lower entries of the filled pattern (= strictly upper)
  // chain: rows nx - chain_t .. nx - 1, each alone in its level in both
  // directions; solved and factorised sequentially in registers
  int chain_t = 0;
  std::vector<int> chain_pos;  // [chain_t][chain_t] positions in the filled pattern, -1 absent

  // Level-sliced schedules (see Sched): the reduction's solves (S = 1024 /
  // col_tile slots), the single-column solves of the step and the
  // refactorisation items (S = threads per scenario group: 64 when the
  // scenario's data sits in LDS, 1024 otherwise).
  Sched red_up, red_dn, stp_up, stp_dn, fac;
  std::vector<int> upd_dst;  // refactorisation update targets (see build_fac_sched)
  int group = 64;            // threads per scenario in the refactorisation
  int step_group = 64;       // threads per scenario in the step's sweeps
  int spw = 1;               // scenarios per workgroup in those kernels (LDS mode)
  bool upd_lds = true;       // LDS refactorisation stages its update targets
  int variant = 1;           // reduction: 1 adjoint solves, 2 stacked product
  int nu_pad = 0;            // row pitch of the stacked panels (multiple of 32)
  int nchunk = 1;            // contraction chunks of the stacked product
};

// Returns an empty string on success, else the error message.
std::string build_symbolic(const rkkt_network& net, int n_scen, const rkkt_options* opt, Sym& s);

// sizes fixing the LDS layouts, for a tile width
LdsSizes lds_sizes(const Sym& s, int w, int variant, int spw);

}  // namespace rkkt

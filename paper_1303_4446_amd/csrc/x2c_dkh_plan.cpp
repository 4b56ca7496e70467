// Host-side plan of the DKHn Hamiltonian: which commutator products are
// formed, into which buffers, with which weights (see x2c_dkh_plan.h).
#include "x2c_dkh_plan.h"

#include <array>

namespace x2c {

namespace {

constexpr int EVEN = 0, ODD = 1;
constexpr int BU = 1, BL = 2, BO = 1;   // even: upper / lower block; odd: upper-right block

// A_i = ad_W^i(part) of the chain started by the part (l, par) at step k;
// it has order l + i k and parity par + i.
struct Node {
  int k, l, par, i, order, npar;
  int need;   // blocks of A_i that are formed
};

double factorial(int i) {
  double f = 1.0;
  for (int j = 2; j <= i; ++j) f *= j;
  return f;
}

int popcount2(int m) { return (m & 1) + ((m >> 1) & 1); }

}  // namespace

bool dkh_plan(int n, DkhPlan& P) {
  if (n < 1 || n > DKH_MAX_ORDER) return false;
  P = DkhPlan();
  P.order = n;
  const int K = n / 2;   // steps k > n/2 change no even term of order <= n
  auto slot_eu = [n](int l) { return l - 1; };
  auto slot_el = [n](int l) { return n + l - 1; };
  auto slot_od = [n](int l) { return 2 * n + l - 1; };
  const int TA_U = 3 * n, TA_L = 3 * n + 1, TB_U = 3 * n + 2, TB_L = 3 * n + 3;
  P.slot_p = 3 * n + 4;
  P.slot_w = 3 * n + 5;
  P.nslot = 3 * n + 6;

  // forward: the chains of every step, sources in descending order (a
  // chain writes only to orders above its source, so the sources of a step
  // are all read before they can change)
  std::vector<std::array<bool, 2>> exist(n + 1, {false, false});
  exist[1] = {true, true};
  std::vector<std::vector<Node>> steps(K + 1);
  for (int k = 1; k <= K; ++k) {
    std::vector<std::array<bool, 2>> add(n + 1, {false, false});
    for (int l = n; l >= 1; --l)
      for (int par : {ODD, EVEN}) {
        if (!exist[l][par]) continue;
        int p = par;
        for (int i = 1; l + i * k <= n; ++i) {
          p = 1 - p;
          steps[k].push_back(Node{k, l, par, i, l + i * k, p, 0});
          add[l + i * k][p] = true;
        }
      }
    for (int j = 1; j <= n; ++j)
      for (int p = 0; p < 2; ++p)
        if (add[j][p]) exist[j][p] = true;
    exist[k][ODD] = false;   // removed by W_k
  }

  // backward: blocks needed of every term after every step, and of every node
  std::vector<std::vector<std::array<int, 2>>> need(K + 1, std::vector<std::array<int, 2>>(n + 1, {0, 0}));
  for (int j = 1; j <= n; ++j) need[K][j][EVEN] = BU;
  std::vector<bool> step_used(K + 1, false);
  for (int k = K; k >= 1; --k) {
    auto prev = need[k];
    prev[k][ODD] = 0;
    auto& nodes = steps[k];
    // chains are contiguous runs of nodes with the same (l, par), i ascending
    size_t s = 0;
    while (s < nodes.size()) {
      size_t e = s;
      while (e < nodes.size() && nodes[e].l == nodes[s].l && nodes[e].par == nodes[s].par) ++e;
      int req = 0;
      for (size_t x = e; x-- > s;) {
        Node& nd = nodes[x];
        const int valid = nd.npar == EVEN ? (BU | BL) : BO;
        const int blocks = (need[k][nd.order][nd.npar] | req) & valid;
        nd.need = blocks;
        req = blocks ? (nd.npar == EVEN ? BO : (BU | BL)) : 0;
        if (blocks) step_used[k] = true;
      }
      prev[nodes[s].l][nodes[s].par] |= req;
      s = e;
    }
    if (step_used[k]) prev[k][ODD] |= BO;
    need[k - 1] = prev;
  }

  // emission
  std::vector<int> inited(P.nslot, 0);
  inited[slot_eu(1)] = inited[slot_el(1)] = inited[slot_od(1)] = 1;   // E_1, E_1', O_1 from the fpFW blocks
  auto term_slot = [&](int order, int par, int blk) {
    if (par == ODD) return slot_od(order);
    return blk == BU ? slot_eu(order) : slot_el(order);
  };
  for (int k = 1; k <= K; ++k) {
    if (!step_used[k]) continue;
    P.ops.push_back(DkhOp{DK_WGEN, slot_od(k), P.slot_w, 0, 0.0, 0});
    const auto& nodes = steps[k];
    size_t s = 0;
    while (s < nodes.size()) {
      size_t e = s;
      while (e < nodes.size() && nodes[e].l == nodes[s].l && nodes[e].par == nodes[s].par) ++e;
      const int l = nodes[s].l, par = nodes[s].par;
      int pu = par == ODD ? slot_od(l) : slot_eu(l), pl = par == ODD ? -1 : slot_el(l);
      for (size_t x = s; x < e; ++x) {
        const Node& nd = nodes[x];
        if (!nd.need) break;   // nothing later in the chain is needed either
        const int cu = (nd.i & 1) ? TA_U : TB_U, cl = (nd.i & 1) ? TA_L : TB_L;
        if (nd.npar == EVEN) {
          if (nd.need & BU) P.ops.push_back(DkhOp{DK_EVEN_U, pu, cu, 0, 0.0, 0});
          if (nd.need & BL) P.ops.push_back(DkhOp{DK_EVEN_L, pu, cl, 0, 0.0, 0});
          P.products += popcount2(nd.need);
        } else {
          P.ops.push_back(DkhOp{DK_ODD, pu, pl, cu, 0.0, 0});
          P.products += 2;
        }
        const double coef = (par == ODD && l == k) ? nd.i / factorial(nd.i + 1) : 1.0 / factorial(nd.i);
        const int keep = nd.need & need[k][nd.order][nd.npar];
        for (int blk : {BU, BL}) {
          if (!(keep & blk)) continue;
          const int src = (nd.npar == ODD || blk == BU) ? cu : cl;
          const int dst = term_slot(nd.order, nd.npar, blk);
          P.ops.push_back(DkhOp{DK_ACC, src, dst, 0, coef, inited[dst]});
          inited[dst] = 1;
        }
        pu = cu;
        pl = cl;
      }
      s = e;
    }
  }
  for (int l = 1; l <= n; ++l)
    if (inited[slot_eu(l)]) P.final_slots.push_back(slot_eu(l));
  P.ops.push_back(DkhOp{DK_FINAL, 0, 0, 0, 0.0, 0});
  return true;
}

}  // namespace x2c

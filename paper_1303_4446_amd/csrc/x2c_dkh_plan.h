// Host-side plan of the DKHn Hamiltonian (exponential parametrisation).
//
// The fpFW Hamiltonian H^0 = D_0 + H_1 (D_0 = diag(E_0 - c^2, -E_0 - c^2))
// is transformed by U_k = exp(W_k), k = 1 .. floor(n/2), with the odd
// anti-Hermitian W_k = [[0, W_k], [-W_k^H, 0]], W_k = O_k / (E_0i + E_0j)
// (Sec. II, "The DKH approach"; later steps change no even term of order
// <= n).  Every term of order l <= n of the current Hamiltonian has an even
// part (upper block E_l, lower block E_l') and an odd part (upper-right O_l).
// Step k replaces H by sum_i ad_W^i(H) / i!, term by term: the chain
// A_0 = part, A_i = [W, A_{i-1}] adds A_i / i! to order l + i k (for the odd
// part of order k the chain of D_0 is folded in: [W, D_0] = -O_k, so O_k
// leaves and ad^i(O_k) enters with weight i / (i+1)!).
//
// The plan keeps only what reaches the n-th order electronic Hamiltonian
// sum_l E_l: a block of a chain node is formed only if a later product or a
// kept term needs it (working backwards from the upper blocks of the final
// even terms), and the Hermitian structure is used as the paper describes:
// [W, odd O] has the upper block W O^H + (W O^H)^H and the lower block
// -(W^H O + (W^H O)^H), one multiplication each; [W, even (E, E')] has the
// upper-right block W E' - E W, two multiplications.  The number of
// multiplications of the plan is P(n) of Table I.
//
// Buffers are slots 0 .. nslot-1: E_l in slot l-1, E_l' in n+l-1, O_l in
// 2n+l-1 (l = 1..n); then two chain nodes (upper / odd, lower) in ping-pong,
// the product scratch and W.
#pragma once

#include <vector>

namespace x2c {

enum DkhOpKind : int {
  DK_WGEN = 0,    // W <- O[a] / (E_0i + E_0j)
  DK_EVEN_U,      // P <- W O[a]^H;  X[b] <- P + P^H           (1 multiplication)
  DK_EVEN_L,      // P <- W^H O[a];  X[b] <- -(P + P^H)        (1 multiplication)
  DK_ODD,         // X[c] <- W E'[b] - E[a] W                 (2 multiplications)
  DK_ACC,         // X[b] <- init ? X[b] + coef X[a] : coef X[a]
  DK_FINAL,       // h <- diag(E_0 - c^2) + sum of the slots a listed in `srcs`
};

struct DkhOp {
  int kind;
  int a, b, c;    // slots
  double coef;
  int init;       // DK_ACC: the destination already holds a value
};

struct DkhPlan {
  int order = 0;
  int nslot = 0;
  int products = 0;             // 2c matrix multiplications (Table I's P(n))
  int slot_w = 0, slot_p = 0;
  std::vector<DkhOp> ops;
  std::vector<int> final_slots; // E_l slots summed into h
};

constexpr int DKH_MAX_ORDER = 14;
constexpr int DKH_MAX_SLOTS = 3 * DKH_MAX_ORDER + 6;

// Builds the plan for 1 <= order <= DKH_MAX_ORDER; false otherwise.
bool dkh_plan(int order, DkhPlan& plan);

}  // namespace x2c

// Host-only parts of the library, with no HIP dependency: scenario-tree
// validation (section 4.1, Fig. 1), checks of the problem data, the offline
// factorisation of Alg. 1 in FP64, ||L|| from the block-diagonal structure of
// L (remark after its definition in section 5.2), the exact nested AV@R cost
// of a trajectory (section 4.2, eq. original-problem) and the work-item list
// of the dataflow sweeps. Built into libspock.so and, on its own, into a CPU
// driver run under AddressSanitizer and UndefinedBehaviorSanitizer.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "../../include/spock.h"

namespace spk {

struct Tree {
  int nn = 0, nl = 0, N = 0;
  std::vector<int> anc, fc, nch, stage;
  std::vector<int> stage_off;  // [N+2]: nodes of stage t are [stage_off[t], stage_off[t+1])
  std::vector<double> prob, pcond;
};

// Builds and validates a tree from breadth-first ancestors and node
// probabilities. Returns SPOCK_OK, SPOCK_EINVAL, SPOCK_ETREE or SPOCK_EPROB.
int build_tree(int32_t nn, const int32_t* anc, const double* prob, Tree& T);

// Finite data, positive weights, ordered boxes, a in [0, 1]. Returns SPOCK_OK,
// SPOCK_EINVAL or SPOCK_EBOX (dimensions are checked by the caller).
int check_problem_data(const Tree& T, const spock_problem_data& d);

// Alg. 1 in FP64, stage N-1 down to 0 (nodes of a stage in parallel): per
// nonleaf node the inverse of R~ and K, per child Abar = A + B K, per node P,
// and per nonleaf node W = sum_c Abar^c' P^c B^c. Row-major per node:
// Abar [nn][nx][nx], K [nl][nu][nx], Rinv [nl][nu][nu], W [nl][nx][nu],
// P [nn][nx][nx]. Returns SPOCK_OK or SPOCK_EFACTOR.
struct Factor {
  std::vector<double> P, Abar, K, Rinv, W;
};
int factor_alg1(const Tree& T, const spock_problem_data& d, Factor& F);

// ||L|| as the largest spectral norm of its blocks (closed forms per block).
double norm_L_blocks(const Tree& T, const spock_problem_data& d);

// Exact nested AV@R cost of (x, u) ([nn][nx], [nl][nu] row-major): leaves
// x'Q_N x; each nonleaf node the AV@R of its children's stage cost plus cost
// to go, with conditional probabilities.
double nested_cost(const Tree& T, int nx, int nu, const double* q, const double* r, const double* qN,
                   const double* a_risk, const std::vector<double>& x, const std::vector<double>& u);

// Work items of the dataflow sweeps with nc children per chunk: backward
// items (families in reverse breadth-first order, chunks in increasing
// order), then forward items (breadth-first); item code = family * chunk_codes
// + chunk. pbase[i] is the first partial-sum slot of a family with several
// chunks; nslots the number of slots. Returns SPOCK_OK, or SPOCK_EINVAL when a
// family needs chunk_codes chunks or more.
int build_flow_items(const Tree& T, int nc, int chunk_codes, std::vector<int>& items, std::vector<int>& pbase,
                     int& nslots, int& nbwd);

// Dense costs (spock_problem_data Qm, Rm, QNm): finite and symmetric, Q and
// Q_N positive semidefinite, R positive definite (cyclic Jacobi
// eigenvalues). Returns SPOCK_OK or SPOCK_EINVAL.
int check_dense_costs(const Tree& T, const spock_problem_data& d);
// Their symmetric square roots V diag(sqrt(lambda)) V', row-major per node:
// Qh, QNh [nn][nx][nx], Rh [nn][nu][nu].
void dense_cost_roots(const Tree& T, const spock_problem_data& d, std::vector<double>& Qh, std::vector<double>& Rh,
                      std::vector<double>& QNh);

// Blocks of the node-parallel post-pass: families packed in breadth-first
// order, block b owning families [bfam[b], bfam[b + 1]) whose children (one
// contiguous run) number at most cap (a family with more children than cap
// gets a block of its own; cap must be at least the largest family for the
// kernel, which the caller checks). Returns the number of blocks.
int build_post_blocks(const Tree& T, int cap, std::vector<int>& bfam);

// General problems (conic risk of section 4.3, polyhedral constraints of
// section 4.1): the vector layout, and per nonleaf node the projector of
// its (y, tau, s) block on S2 = ker [E' -I -I; F' 0 0] (FP64, row-major
// m x m, m = ny + 2 n_i), I - G'(G G')^+ G from an eigendecomposition of
// G G'. Offsets: z2off[i] of the (y, tau, s) block in z, e1off[i] of group
// 1 (y, s-row, nc constraint rows) in eta, Eoff / yoff / Poff of node i's
// E, b and projector in their concatenations.
struct GeneralLayout {
  int nc = 0, ncN = 0;
  long long nz = 0, neta = 0, eE2 = 0, eE3 = 0;
  std::vector<int> ny, nnu, kpos;                      // [nl]
  std::vector<long long> z2off, e1off, Eoff, yoff, Poff;  // [nl]
  std::vector<double> E, b, PS2;
};
// Validates the risk and constraint data of d (either may be NULL: AV@R
// from a_risk, or the boxes) and builds the layout. max_block bounds
// ny + 2 n_i. Returns SPOCK_OK, SPOCK_EINVAL, SPOCK_EBOX or
// SPOCK_EUNSUPPORTED.
int build_general(const Tree& T, const spock_problem_data& d, int max_block, GeneralLayout& G);
// ||L|| of a general problem: the largest spectral norm of its blocks
// ((x^i, u^i): Gamma' Gamma + sum_c diag(q^c, r^c); (y^i, s^i): closed form in
// ||b^i||; tau^c and leaf s^j: 1/2; leaf x^j: Gamma_N' Gamma_N + diag(q_N)).
double norm_L_general(const Tree& T, const spock_problem_data& d, const GeneralLayout& G);
// Largest eigenvalue of a symmetric k x k matrix (row-major; cyclic Jacobi).
double sym_max_eig(int k, std::vector<double> A);

// Parallel loop over [0, n) on up to 16 host threads.
template <typename F>
void parallel_for(int n, F&& f) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::min<unsigned>(hw ? hw : 1, 16u);
  if (n < 64 || nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  nt = std::min(nt, n);
  std::vector<std::thread> th;
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w]() {
      for (int i = w; i < n; i += nt) f(i);
    });
  for (auto& t : th) t.join();
}

}  // namespace spk

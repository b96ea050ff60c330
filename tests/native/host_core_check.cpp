// CPU driver of the host-only library code (host_core.cpp) for the sanitizer
// test: reads one case from a text file (argv[1]) and prints what the
// library computes, one labelled array per line, for the test to compare
// with the oracle. Input (whitespace-separated): nn nx nu; anc[nn];
// prob[nn]; A B q r qN xmin xmax umin umax a_risk (the spock_problem_data
// arrays); x[nn][nx] u[nl][nu] (a trajectory); nc (children per chunk);
// dense (0 or 1), then, if 1, Qm[nn][nx][nx] Rm[nn][nu][nu] QNm[nn][nx][nx]
// (dense costs: their check, their symmetric roots and ||L|| of the general
// layout are printed in place of the diagonal figures).
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <algorithm>
#include <vector>

#include "../../paper_2212_01110_amd/csrc/host_core.h"

using spk::Tree;

static void put(const char* name, const std::vector<double>& v) {
  std::printf("%s", name);
  for (double x : v) std::printf(" %.17g", x);
  std::printf("\n");
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  std::ifstream in(argv[1]);
  int nn = 0, nx = 0, nu = 0;
  in >> nn >> nx >> nu;
  std::vector<int32_t> anc(nn);
  std::vector<double> prob(nn);
  for (auto& a : anc) in >> a;
  for (auto& p : prob) in >> p;
  // tokens through strtod, which also reads inf and nan
  auto read = [&](size_t n) {
    std::vector<double> v(n);
    std::string tok;
    for (auto& x : v) {
      in >> tok;
      x = std::strtod(tok.c_str(), nullptr);
    }
    return v;
  };
  std::vector<double> A = read((size_t)nn * nx * nx), B = read((size_t)nn * nx * nu), q = read((size_t)nn * nx),
                      r = read((size_t)nn * nu), qN = read((size_t)nn * nx), xmin = read((size_t)nn * nx),
                      xmax = read((size_t)nn * nx), umin = read((size_t)nn * nu), umax = read((size_t)nn * nu),
                      a = read(nn);
  Tree T;
  const int rt = spk::build_tree(nn, anc.data(), prob.data(), T);
  std::printf("tree_rc %d\n", rt);
  if (rt != SPOCK_OK) return 0;
  std::printf("shape %d %d %d\n", T.N, T.nl, T.nn - T.nl);
  std::vector<double> x = read((size_t)nn * nx), u = read((size_t)T.nl * nu);
  int nc = 1, dense = 0;
  in >> nc >> dense;
  std::vector<double> Qm, Rm, QNm;
  if (dense) {
    Qm = read((size_t)nn * nx * nx);
    Rm = read((size_t)nn * nu * nu);
    QNm = read((size_t)nn * nx * nx);
  }
  spock_problem_data d{};
  d.nx = nx;
  d.nu = nu;
  d.A = A.data();
  d.B = B.data();
  d.q = q.data();
  d.r = r.data();
  d.qN = qN.data();
  d.xmin = xmin.data();
  d.xmax = xmax.data();
  d.umin = umin.data();
  d.umax = umax.data();
  d.a_risk = a.data();
  if (dense) {
    d.Qm = Qm.data();
    d.Rm = Rm.data();
    d.QNm = QNm.data();
  }
  const int rd = spk::check_problem_data(T, d);
  std::printf("data_rc %d\n", rd);
  if (rd != SPOCK_OK) return 0;
  if (dense) {
    std::vector<double> Qh, Rh, QNh;
    spk::dense_cost_roots(T, d, Qh, Rh, QNh);
    put("Qh", Qh);
    put("Rh", Rh);
    put("QNh", QNh);
    spk::GeneralLayout GL;
    const int rg = spk::build_general(T, d, 96, GL);  // the library's block bound
    std::printf("general_rc %d\n", rg);
    if (rg == SPOCK_OK) std::printf("normL %.17g\n", spk::norm_L_general(T, d, GL));
    return 0;
  }
  spk::Factor F;
  const int rf = spk::factor_alg1(T, d, F);
  std::printf("factor_rc %d\n", rf);
  if (rf != SPOCK_OK) return 0;
  put("K", F.K);
  put("Abar", F.Abar);
  put("P", F.P);
  put("Rinv", F.Rinv);
  put("W", F.W);
  std::printf("normL %.17g\n", spk::norm_L_blocks(T, d));
  std::printf("nested %.17g\n", spk::nested_cost(T, nx, nu, q.data(), r.data(), qN.data(), a.data(), x, u));
  std::vector<int> items, pbase;
  int nslots = 0, nbwd = 0;
  const int ri = spk::build_flow_items(T, nc, 64, items, pbase, nslots, nbwd);
  std::printf("items_rc %d %d %d\n", ri, nbwd, nslots);
  std::vector<double> it(items.begin(), items.end());
  put("items", it);
  // post-pass blocks at the capacities the library uses (teams per block
  // 32, 16, 8, 4, raised to the largest family)
  int maxnch = 1;
  for (int i = 0; i < T.nl; ++i) maxnch = std::max(maxnch, T.nch[i]);
  for (int tpb : {32, 16, 8, 4}) {
    std::vector<int> bf;
    const int cap = std::max(tpb, maxnch);
    const int nb = spk::build_post_blocks(T, cap, bf);
    std::printf("pblk%d %d %d\n", tpb, nb, cap);
    std::vector<double> b(bf.begin(), bf.end());
    put(("pblk" + std::to_string(tpb) + "_f").c_str(), b);
  }
  return 0;
}

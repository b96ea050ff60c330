// Internal structures shared by the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>
#include <string>

#include "../../include/spock.h"
#include "host_core.h"

namespace spk {

// Maximum state/input dimension handled by the team kernels.
constexpr int kMaxDim = 64;
// Number of FP64 statistics produced per block of the forward sweep:
// sum r_z^2, sum r_eta^2, sum r_eta.(L r_z), max |xi_p|, max |xi_d|.
constexpr int kStats = 5;
// Mapping code of the workgroup-per-family kernels.
constexpr int kTeamWG = 256;
// Mapping code of the one-launch dataflow form of T (flow.hip).
constexpr int kTeamFlow = 512;
// Mapping code reported by the shared-tree batched form (shared.hip).
constexpr int kTeamShared = 1024;

// Device view of one problem's iteration data in precision S. Node-indexed
// arrays follow breadth-first order; matrices are stored as the transpose of
// the operator they feed ("input-major"): element (out o, in k) at k*nout+o,
// so a team of lanes, one lane per output, reads contiguous memory.
template <typename S>
struct DevProb {
  int nn, nl, nx, nu, N;
  long long nz, neta;
  long long zU, zZ2;   // z offsets: first u, first z2 block
  long long eE2, eE3;  // eta offsets: first group-2 block, first group-3 block
  const int* fc;       // first child (nonleaf), -1 at leaves
  const int* nch;      // number of children
  const int* anc;
  const S* p;          // conditional probability of the node given its ancestor
  const S* a;          // AV@R a of nonleaf nodes
  const S* sq;         // [nn][nx] sqrt(diag Q^c)
  const S* sr;         // [nn][nu] sqrt(diag R^c)
  const S* sqN;        // [nn][nx] sqrt(diag Q_N^j)
  const S* xlo; const S* xhi;  // [nn][nx]
  const S* ulo; const S* uhi;  // [nn][nu]
  const S* AbR;  // [nn][nx][nx]  Abar^c row-major      (Abar' q, backward)
  const S* AbC;  // [nn][nx][nx]  Abar^c column-major   (Abar x, forward)
  const S* BR;   // [nn][nx][nu]  B^c row-major         (B' q, backward)
  const S* BC;   // [nn][nu][nx]  B^c column-major      (B d, forward)
  const S* KR;   // [nl][nu][nx]  K row-major           (K' e, backward)
  const S* KC;   // [nl][nx][nu]  K column-major        (K x, forward)
  const S* Rinv; // [nl][nu][nu]  inverse of R~ (symmetric)
  const S* WC;   // [nl][nu][nx]  W = sum_c Abar'P B, column-major (W d, backward)
  const S* M1C;  // [nl][nu][nx]  M1 = (K' + W) R~^{-1}, column-major (per-stage forms)
  // backward step of the dataflow form in one mat-vec phase (FP64-formed):
  //   d = R~^{-1} ubar + sum_c Bt^c q^c,  q = P1 ubar - xbar + sum_c At^c q^c
  const S* AtR;  // [nn][nx][nx]  At^c = Abar^c' - M1 B^c' (parent's M1), stored like AbR's role
  const S* BtR;  // [nn][nx][nu]  Bt^c = -R~^{-1} B^c' (parent's R~^{-1}), stored like BR's role
  const S* P1C;  // [nl][nu][nx]  P1 = M1 - K', stored like M1C
  S alpha;
};


// Device view of the general parts of a problem (conic risk of section 4.3,
// polyhedral constraints of section 4.1), precision S. Per nonleaf node i:
// z2off[i] the offset in z of its block (y^i, tau of its children, s of its
// children); e1off[i] the offset in eta of its group 1 (y^i, s^i - b'y^i,
// the nc constraint rows); ny, kpos; E^i [ny][n_i] row-major at E + Eoff[i];
// b^i at b + yoff[i]; the S2 projector of its (y, tau, s) block (m x m,
// m = ny + 2 n_i, row-major) at PS2 + Poff[i]; Gx [nl][nc][nx],
// Gu [nl][nc][nu], cmin, cmax [nl][nc]. Per leaf j (index j - nl):
// GN [nleaf][ncN][nx], cNmin, cNmax [nleaf][ncN]. Group 2 of non-root c at
// eE2 + (c - 1)(nx + nu + 2); group 3 of leaf j at eE3 + (j - nl)(ncN + nx + 2).
template <typename S>
struct GenDev {
  int nc = 0, ncN = 0;
  long long eE2 = 0, eE3 = 0;
  const long long* z2off = nullptr;
  const long long* e1off = nullptr;
  const int* ny = nullptr;
  const int* kpos = nullptr;
  const long long* Eoff = nullptr;
  const long long* yoff = nullptr;
  const long long* Poff = nullptr;
  const S* E = nullptr;
  const S* b = nullptr;
  const S* PS2 = nullptr;
  const S* Gx = nullptr;
  const S* Gu = nullptr;
  const S* cmin = nullptr;
  const S* cmax = nullptr;
  const S* GN = nullptr;
  const S* cNmin = nullptr;
  const S* cNmax = nullptr;
  // dense costs: symmetric square roots of Q^c, R^c, Q_N^j, row-major per
  // node ([nn][nx][nx], [nn][nu][nu], [nn][nx][nx]); nullptr: the diagonal
  // roots sq, sr, sqN of the problem
  const S* Qh = nullptr;
  const S* Rh = nullptr;
  const S* QNh = nullptr;
};

// Device arrays of one precision.
struct DevArrays {
  void* base = nullptr;  // one allocation holding everything below
  size_t bytes = 0;
};

// Device state of the dataflow form of the sweeps: the tagged exchange
// buffers (q, d of the backward step, x of the forward step; 64-bit words
// holding the launch epoch and half of a value, zeroed once and never
// cleared) and an error word raised by a bounded poll that gave up.
constexpr int kChunkCodes = 64;  // item code = family * kChunkCodes + chunk (chunks per family < 64)
struct FlowState {
  void* mem = nullptr;
  unsigned* err = nullptr;          // [1]
  unsigned long long* qt = nullptr;  // [nl][nx][words per element]
  unsigned long long* dt = nullptr;  // [nl][nu][...]
  unsigned long long* xt = nullptr;  // [nn][nx][...]
  unsigned long long* pt = nullptr;  // [slots][nx + nu][...] partial sums of backward chunks
  int* items = nullptr;              // family * kChunkCodes + chunk; backward, then forward
  int* pbase = nullptr;              // [nl] first partial slot of a family with several chunks
  int nbwd = 0;                      // backward items (as many forward items follow)
  int nc = 1;                        // children per LDS chunk
  int grid = 0;                      // workgroups launched (0: form unavailable)
  int resident = 0;                  // resident capacity the grid is bounded by
  unsigned spin = 1u << 21;          // polls of one bounded wait before it gives up
  int occ = 5;                       // register budget: 4 to 7 wavefronts per SIMD
  int elem = 0;                      // element size the state was sized for
  int budget = 32 * 1024;            // LDS budget the chunk size was chosen for
  // cooperative launch (residency guaranteed by the runtime) or a plain
  // launch of the resident-sized grid (about 20 us less dispatch per T; a
  // grid that were not all resident ends with the error word set)
  bool coop = false;
};

// Statistics of one evaluation of T handed to the host without a copy: the
// last kernel writes them into pinned, coherent host memory and then the
// epoch of the evaluation into flag (system-scope release); the host polls
// the flag.
struct Mailbox {
  double v[8];
  unsigned long long flag;
  unsigned long long pad[7];
};
struct Publish {
  Mailbox* mb = nullptr;  // device view of the mailbox (nullptr: no publish)
  unsigned long long epoch = 0;
};

struct Problem {
  const Tree* tree = nullptr;
  int precision = SPOCK_FP64;
  int nx = 0, nu = 0;
  long long nz = 0, neta = 0;
  double alpha = 0, normL = 0;
  // host copies needed by the solver (box of the root, nested cost)
  std::vector<double> xlo0, xhi0;
  std::vector<double> q, r, qN, a_risk;  // for the nested cost
  // device
  void* dmem = nullptr;
  int* d_fc = nullptr; int* d_nch = nullptr; int* d_anc = nullptr;
  int* d_stage_off = nullptr;
  DevProb<double> dp64{};
  DevProb<float> dp32{};
  // per-problem work buffers (allocated lazily, precision-sized)
  void* work = nullptr;
  size_t work_bytes = 0;
  // lanes per family: 8, 16, 32 or 64 (team kernels), or kTeamWG for one
  // 256-thread workgroup per family
  int team = 64;
  int teams_per_block = 4;
  // first stage walked by subtree-owning workgroups (workgroup mapping only);
  // N means every stage has its own launch
  int cut = 0;
  int team_pp = 64;  // lanes per family of the parallel pre/post passes
  // node-parallel post-pass, per team size 8, 16, 32, 64 (index log2(T) - 3):
  // the device block table (pblk_n[k] + 1 family indices) and the child
  // capacity of a block; pblk_n[k] = 0 selects the family-serial kernel
  const int* d_pblk[4] = {};
  int pblk_n[4] = {};
  int pblk_cap[4] = {};
  // flat post-pass (one wavefront per family or leaf) in place of the team
  // forms; d_spos [nn]: offset in z of s^c in its ancestor's block (0 at
  // the root)
  bool post_flat = false;
  const long long* d_spos = nullptr;
  int ncu = 256;    // compute units of the device (grid of the flat post-pass)
  int flat_bpc = 1;  // resident blocks of the flat post-pass per compute unit
  bool tuned = false;
  // general conic risk / polyhedral constraints (general kernels for the
  // pre- and post-passes, L, L*, prox of g* and M; device block gmem)
  bool general = false;
  void* gmem = nullptr;
  GenDev<double> gd64{};
  GenDev<float> gd32{};
  // set once a bounded wait of the dataflow sweeps gave up: the problem then
  // runs the per-stage workgroup form for good
  bool flow_failed = false;
  FlowState flow;
  mutable unsigned flow_epoch = 0;  // tag of the last dataflow launch (never 0 once launched)
  // when set, launch_T records prof[0..4] before the pre-pass, after it,
  // after the sweeps, after the post-pass and at the end (timing aid)
  hipEvent_t* prof = nullptr;
  Mailbox* mbox = nullptr;      // host view (hipHostMalloc, coherent)
  Mailbox* mbox_dev = nullptr;  // device view of the same memory
  unsigned long long mbox_epoch = 0;
};

// ---------------------------------------------------------------- launchers
// (kernels.hip) All return hipError_t of the last launch.
// T(v) (or prox_f of z when dual is false): parallel pre-pass, backward and
// forward sweeps, parallel post-pass with the residual statistics.
// Sweep mapping of one launch (team 0: the problem's own mapping and cut).
struct SweepMap {
  int team = 0;
  int cut = 0;
};
template <typename S>
hipError_t launch_T(const Problem& P, const S* v, S* Tv, const double* x0, S* q, S* d, S* xbar,
                    S* ubar, double* partials, double* stats_dev, hipStream_t st,
                    const S* eta_zero, bool dual, Publish pub = Publish{}, SweepMap map = SweepMap{});
int post_blocks(const Problem& P);
int flat_post_blocks(const Problem& P);
int family_wave_blocks(int nl);
template <typename S>
int flat_post_occupancy();
// General problems (general.hip): pre-pass, post-pass with statistics
// (post_blocks records), L, L*, prox of g* and M, one thread per family.
// kGenMaxBlock bounds ny + 2 n_i of a family (its (y, tau, s) block).
constexpr int kGenMaxBlock = 96;
int gen_post_blocks(const Problem& P);
template <typename S>
hipError_t launch_gen_pre(const Problem& P, const S* z, const S* eta, S* zout, S* xbar, S* ubar, S* qbuf,
                          hipStream_t st);
template <typename S>
hipError_t launch_gen_post(const Problem& P, const S* z, const S* eta, const S* zout, S* eout, double* partials,
                           hipStream_t st);
template <typename S>
hipError_t launch_gen_L(const Problem& P, const S* z, S* eta, hipStream_t st);
template <typename S>
hipError_t launch_gen_Lt(const Problem& P, const S* eta, S* z, hipStream_t st);
template <typename S>
hipError_t launch_gen_prox_gstar(const Problem& P, const S* w, S* out, hipStream_t st);
template <typename S>
hipError_t launch_gen_M(const Problem& P, const S* d, S* Md, hipStream_t st);
// Dataflow form of the sweeps (flow.hip): one persistent launch per T.
template <typename S>
hipError_t launch_sweeps_flow(const Problem& P, const DevProb<S>& D, S* zout, const double* x0, const S* xbar,
                              const S* ubar, S* q, S* d, hipStream_t st);
int flow_lds_bytes(int nx, int nu, int nc, int elem);
template <typename S>
const void* flow_kernel(int occ);
template <typename S>
hipError_t launch_L(const Problem& P, const S* z, S* eta, hipStream_t st);
template <typename S>
hipError_t launch_Lt(const Problem& P, const S* eta, S* z, hipStream_t st);
// L and L* of B instances whose vectors are `is` elements apart (special form)
template <typename S>
hipError_t launch_L_batch(const Problem& P, const S* z, S* eta, long long is, int B, hipStream_t st);
template <typename S>
hipError_t launch_Lt_batch(const Problem& P, const S* eta, S* z, long long is, int B, hipStream_t st);
template <typename S>
hipError_t launch_prox_gstar(const Problem& P, const S* w, S* out, hipStream_t st);
// M d = (d_z - alpha L* d_eta, d_eta - alpha L d_z), team of team_pp lanes per family
template <typename S>
hipError_t launch_M(const Problem& P, const S* d, S* Md, hipStream_t st);

// Up to 8 device vectors passed by value to a kernel.
template <typename S>
struct VecPtrs {
  const S* p[8];
};

// Vector kernels for the SuperMann/Anderson layer (FP64 accumulation).
template <typename S>
hipError_t launch_lincomb(long long n, S* out, double a, const S* x, double b, const S* y,
                          hipStream_t st);
template <typename S>
hipError_t launch_lincomb3(long long n, S* out, double a, const S* x, double b, const S* y,
                           double c, const S* w, hipStream_t st);
template <typename S>
hipError_t launch_dots(long long n, int k, VecPtrs<S> xs, VecPtrs<S> ys, double* partials,
                       double* out_dev, hipStream_t st);
// Anderson step on the device: the push about to run (slots of the columns
// before it, oldest first, and the slot of the new column).
struct AAPush {
  int m, mo, slot;
  int order_old[4];
};
// The Anderson ring on the device (memory m <= kAAMax): the column slots in
// use, oldest first, as the last Gram solve left them, and the columns (slots)
// the last direction used. The host sets m and cnt = 0 once per solve.
constexpr int kAAMax = 4;
struct AARingDev {
  int m;
  int cnt;
  int order[kAAMax];
  int dk;
  int dslot[kAAMax];
};
// Grid sums finished inside a vector kernel: tagged records of the blocks
// and of groups of kRedGroup blocks (kRedRecWords 64-bit words, zeroed once;
// every launch's tag differs from the earlier ones' and is not 0) and
// kRedCounters arrival counters (zero between launches).
constexpr int kRedGroup = 32;
constexpr int kRedMaxBlocks = 1024;
constexpr int kRedRecWords = (kRedMaxBlocks + kRedMaxBlocks / kRedGroup) * 16;
constexpr int kRedCounters = kRedMaxBlocks / kRedGroup + 1;
// Push of the newest difference pair into the slot the ring picks (E =
// dV - dR of slot s at eb + s stride, dR at rb + s stride), its Gram row and
// right-hand side (fixed-order sums finished in the launch over the tagged
// records above), then the Gram solve in the last workgroup: gamma for the
// columns of the new order, and the ring updated.
template <typename S>
hipError_t launch_aa_push(long long n, const S* v, const S* vprev, const S* Tv, const S* rprev, S* r_out, S* eb,
                          S* rb, long long stride, unsigned long long* rec, unsigned* counter, unsigned tag,
                          double* G, AARingDev* ring, double* gamma, hipStream_t st);
// d = -r - sum_j gamma_j E_j over the columns of the last push (the ring's
// dk, dslot; E_j = dV_j - dR_j as stored by the push, at eb + slot stride);
// when step is non-null also step = base + d
template <typename S>
hipError_t launch_aa_dir(long long n, const S* r, const S* eb, long long stride, const AARingDev* ring,
                         const double* gamma_dev, S* d, const S* base, S* step, hipStream_t st);
template <typename S>
hipError_t launch_fill(long long n, S* out, double val, hipStream_t st);
// out_i = sum_j c[i][j] in_j, elementwise over n (outputs may alias inputs);
// the vector operations of the QR-updated Anderson step
constexpr int kMixMax = 12;
template <typename S>
struct ColMix {
  int nin = 0, nout = 0;
  const S* in[kMixMax] = {};
  S* out[kMixMax] = {};
  double c[kMixMax][kMixMax] = {};
};
template <typename S>
hipError_t launch_colmix(long long n, const ColMix<S>& M, hipStream_t st);

// Krylov basis of the adjoint GMRES: V_j = basis + j * stride, j < n <=
// kBasisMax. Dots: out_dev[j] = <V_j, x> (FP64), and out_dev[n] = <x, x>
// when xx, also written to host_out (device view of mapped pinned memory)
// when given; part holds (n + 1) * kBasisChunks doubles. Mix: out = a x +
// sum_j C.c[j] V_j (out may be x).
constexpr int kBasisMax = 128;
constexpr int kBasisChunks = 64;
struct BasisCoef {
  double c[kBasisMax];
};
template <typename S>
hipError_t launch_basis_dots(long long nv, int n, const S* basis, long long stride, const S* x, bool xx,
                             double* part, double* out_dev, hipStream_t st, double* host_out = nullptr);
template <typename S>
hipError_t launch_basis_mix(long long nv, int n, const S* basis, long long stride, const BasisCoef& C, double a,
                            const S* x, S* out, hipStream_t st);
// x -= sum_{j < n} c_dev[j] V_j in place; with norm, then x /= sqrt(c_dev[n]
// - sum_j c_dev[j]^2) (0 if that is not positive)
template <typename S>
hipError_t launch_basis_orth(long long nv, int n, const S* basis, long long stride, const double* c_dev, bool norm,
                             S* x, hipStream_t st);
// <v - Tv, w> to *out_dev (fixed-order sum in the last workgroup to finish,
// counted on *counter, over tagged records as for the push), then the
// statistics stats[0..8) published to pub.
template <typename S>
hipError_t launch_rdot(long long n, const S* v, const S* Tv, const S* w, unsigned long long* rec, unsigned* counter,
                       unsigned tag, double* out_dev, const double* stats, Publish pub, hipStream_t st);

int dots_blocks(long long n);


// ---------------------------------------------------------------- batched engine
struct BatchSettings {
  double eps_abs, eps_rel;
  int max_iters, method, m, max_ls;
  double c0, c1, c2, beta, sigma, lambda;
  int write_out;  // 0: leave v_io untouched (timing runs of the autotuner)
};

// One instance of a batched solve (device-resident descriptor).
template <typename S>
struct BatchInst {
  DevProb<S> P;
  const int* stage_off;  // [N+2]
  const double* x0;      // [nx]
  S* vio;                // [n_v] warm start in, T(v^k) out
  S* work;               // pool of vectors + sweep buffers
  long long nv;
};

template <typename S>
hipError_t launch_solve_batched(const BatchInst<S>* insts_dev, int B, const BatchSettings& s, int team,
                                int VM, double* infos_dev, int grid, hipStream_t st);
size_t batched_pool_vectors();

// ---------------------------------------------------------------- adjoint (backward.hip)
template <typename S>
hipError_t launch_jg(const Problem& P, const S* b, const S* w, S* out, hipStream_t st);
template <typename S>
hipError_t launch_jg_batch(const Problem& P, const S* b, const S* w, S* out, long long is, int B, hipStream_t st);
template <typename S>
hipError_t launch_phiT(const Problem& P, const S* cz, S* mu, hipStream_t st);
template <typename S>
hipError_t launch_grad_q(const Problem& P, const S* vstar, const S* la, const S* lb, double* gq,
                         double* gqN, hipStream_t st);
template <typename S>
hipError_t launch_maxdiff(long long n, const S* a, const S* b, double* partials, double* out,
                          hipStream_t st);
template <typename S>
hipError_t launch_copy_elem(S* dst, const S* src, hipStream_t st);

// Shared-tree batched form (shared.hip): B instances of one problem that
// differ in x0 and iterate, in lockstep rounds of one evaluation of T for all
// (MFMA sweeps); results and errors as spock_solve_batched. Keeps a device
// workspace between calls (not thread safe).
template <typename S>
int shared_solve(Problem& P, int B, const double* const* x0, const spock_settings& s, void* const* vio,
                 spock_info* infos, hipStream_t st);
// Adjoint gradients of B instances of one problem at once (the shared-tree
// sweeps for J_f', lockstep GMRES per instance); arguments as spock_backward,
// one per instance.
template <typename S>
int shared_backward(Problem& P, int B, const void* const* vstar, const double* const* x0, double gV,
                    const double* const* gu0, double* const* gx0, double* const* gq, double* const* gqN,
                    const spock_settings& s, spock_info* infos, hipStream_t st);

}  // namespace spk

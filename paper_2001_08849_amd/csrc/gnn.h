// Learned preconditioner: network parameters, per-mesh work buffers and the
// host entry points used by the C ABI.
#pragma once
#include <functional>
#include <memory>

#include "ctx.h"

namespace sfem {

constexpr int kH = 64;        // hidden width
constexpr int kLayers = 4;    // message-passing layers
constexpr int kFNode = 8;     // node input features
constexpr int kFEdge = 12;    // edge input features

// Offsets of the parameter tensors in one flat FP32 vector (row-major
// [fan_out][fan_in] matrices).
struct ParamLayout {
  int64_t Wn, bn, We, be;
  int64_t W[kLayers], b[kLayers], U[kLayers], c[kLayers];
  int64_t Wo;
  int64_t total;
};
const ParamLayout& param_layout();

// Network parameters (FP32 master copy, BF16 copy for the MFMA layers) and
// Adam state.  Lives on one device.
struct Gnn {
  int device = 0;
  std::string err;
  DBuf<float> params, grad, adam_m, adam_v;
  DBuf<__bf16> params_bf16;
  DBuf<float> wpart;             // split-K partial sums of the weight gradients
  int64_t adam_t = 0;
};

// Per-context graph, features, activations, gradients and training pairs.
struct GnnWork {
  const void* graph_for = nullptr;
  int64_t N = 0, nb = 0;
  DBuf<int32_t> erow, etr;       // row node and transposed edge of every edge
  DBuf<float> x, y;              // input features [N][8], [nb][12]
  DBuf<double> s, part;          // d^-1/2 [3N]; reduction partials
  bool have_features = false;
  // forward activations (layer inputs h_l, e_l for l = 0..L; z_l, t_l, a_l)
  DBuf<float> h, e, z, t, a;
  // backward
  DBuf<float> dS, dh, de, dz, dt, da, dXh;
  // training pairs [n_pairs][3N] and K-norms e.K e
  int64_t n_pairs = 0;
  DBuf<float> pr, pe;
  std::vector<double> pden;
  // minibatch panels [3N][B]
  DBuf<float> br, be, bw, bkw, bgh, brh;
  DBuf<int32_t> bidx;
  DBuf<double> bpart;
};

GnnWork& gnn_work(Ctx& c);

// Node and edge features of the context's BC-applied K (requires assembly).
void gnn_features(Ctx& c);
// Forward pass; keep = store every layer's activations (training).  Writes
// S' into c.mval (scalar-CSR layout of K) and d^-1/2 into c.msqrt.
void gnn_forward(Ctx& c, Gnn& g, bool keep);
// Inference: forward, then S' = theta S with theta = min(1, 0.9 / (1.05
// |lambda_min(S)|)) (lambda_min from Lanczos) so that I + S' is positive
// definite; enables the learned preconditioner on the context.
void gnn_precondition(Ctx& c, Gnn& g);
constexpr int kLanczosSteps = 40;
// Loss of the pairs `ids` (host indices) and, with grad, the gradient in
// g.grad (same layout as the parameters).
double gnn_loss_grad(Ctx& c, Gnn& g, const int32_t* ids, int B, bool grad);
void gnn_init_params(Gnn& g, uint64_t seed);
void gnn_adam(Gnn& g, hipStream_t s, double lr, double beta1, double beta2, double eps);
// Training pairs from Jacobi-PCG runs on the context's K: run k solves
// K x = b_k (b_0 = the load, others seeded random loads) and stores
// (r, e) = (K (x* - x_j), x* - x_j) for snapshots x_j spread over the run.
int64_t gnn_generate_pairs(Ctx& c, int n_rhs, int snaps_per_rhs, uint64_t seed);
void gnn_set_pairs(Ctx& c, int64_t n_pairs, const float* r, const float* e);

// solve.hip: Jacobi PCG (FP64) of K x = b from x = 0 to ||b - K x|| <=
// tol_abs; hook(done) runs after every check period of at most `every`
// iterations with c.x current; a period also ends at next_stop(done) when
// that is sooner (next_stop may be null).
int jacobi_run(Ctx& c, const double* b, double tol_abs, int every, int max_iter,
               const std::function<void(int)>& hook,
               const std::function<int(int)>* next_stop = nullptr);
// z = M r with the learned preconditioner (FP64 vectors).
void learned_apply(Ctx& c, const double* r, double* z);

}  // namespace sfem

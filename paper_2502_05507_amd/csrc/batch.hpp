// Engine behind the batched (bae_batch_*) and served (bae_server_*) solves: member
// problems share one set of launches per GMRES phase and advance independently.
#pragma once

#include <vector>

#include "context.hpp"

namespace bae {

struct BatchEngine;

BatchEngine* batch_engine_new(int device, hipStream_t stream);
void batch_engine_delete(BatchEngine* b);
// New member list: rebuilds descriptors and work lists (members keep their GMRES state).
void batch_set_members(BatchEngine* b, const std::vector<bae_ctx*>& members);
// Start GMRES on the masked members from r0 = b (sel 0) or r (sel 1).
void batch_begin(BatchEngine* b, const std::vector<int32_t>& mask, int sel, const std::vector<double>& tol,
                 const std::vector<int>& maxit);
// `iters` iterations of every unfinished member.
void batch_iterate(BatchEngine* b, int prec, int iters, bool use_graph);
std::vector<int32_t> batch_done(BatchEngine* b);
std::vector<int32_t> batch_kdone(BatchEngine* b);
// x (+)= V y on the masked members.
void batch_finish(BatchEngine* b, const std::vector<int32_t>& mask, bool accumulate);
// x = 0 (mode 1) or r = b (mode 2) on the masked members.
void batch_vec(BatchEngine* b, int mode, const std::vector<int32_t>& mask);
std::vector<double> batch_bnorms(BatchEngine* b);
// r = b - A64 x; ||r|| per member (all members, or the masked ones).
std::vector<double> batch_residual_norms(BatchEngine* b, const std::vector<int32_t>* mask);
// u_gamma = D x + u_p for all members (or the masked ones).
void batch_gamma_values(BatchEngine* b, const std::vector<int32_t>* mask);
std::vector<double> batch_history(BatchEngine* b, int p, int count);

}  // namespace bae

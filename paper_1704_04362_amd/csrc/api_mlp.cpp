// C ABI of the learned lateral-leverage proposal (features, forward pass,
// training step, sampling weights). Validation and kernel order only.
#include <cmath>
#include <string>

#include "common.hpp"
#include "mlp.hpp"

namespace tp {
namespace {
hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int check_a(const tp_tensor* A) {
  if (!A || !A->data) return fail(TP_EINVAL, "A is null");
  if (A->dtype != TP_F32) return fail(TP_EDTYPE, "features need float32 data");
  if (A->n1 < 1 || A->n2 < 2 || A->n3 < 4 || A->n3 % 4) return fail(TP_ESHAPE, "need n1 >= 1, n2 >= 2, n3 % 4 == 0");
  return TP_OK;
}
}  // namespace
}  // namespace tp

using namespace tp;

extern "C" {

int tp_mlp_param_count(void) { return kMlpParams; }

size_t tp_mlp_features_workspace(const tp_tensor* A) {
  if (!A) return 0;
  return mlp_features_ws(A->n1, A->n2);
}

int tp_mlp_features(const tp_tensor* A, const float* phi, float* feat, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_a(A)) return rc;
  if (!phi || !feat) return fail(TP_EINVAL, "phi / feat are null");
  if (!ws || ws_bytes < tp_mlp_features_workspace(A)) return fail(TP_EWORKSPACE, "feature workspace too small");
  return mlp_features((const float*)A->data, A->n1, A->n2, A->n3, phi, feat, ws, S(stream));
}

int tp_mlp_forward(const float* params, const float* feat, int64_t nrows, float* logits, void* stream) {
  if (!params || !feat || !logits) return fail(TP_EINVAL, "null pointer");
  if (nrows < 0) return fail(TP_EINVAL, "nrows < 0");
  return mlp_forward(params, feat, nrows, logits, S(stream));
}

size_t tp_mlp_train_workspace(int64_t ntensors, int64_t nslices) {
  if (ntensors < 1 || nslices < 1) return 0;
  return mlp_train_ws(ntensors, nslices);
}

int tp_mlp_train_step(float* params, float* m, float* v, int64_t step, double lr, const float* feat,
                      const float* target, int64_t ntensors, int64_t nslices, float* loss, float* grad, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!params || !feat || !target) return fail(TP_EINVAL, "null pointer");
  if (step > 0 && (!m || !v)) return fail(TP_EINVAL, "Adam moments are null");
  if (ntensors < 1 || nslices < 1) return fail(TP_EINVAL, "need at least one tensor and one slice");
  if (step < 0 || !(lr >= 0.0) || !std::isfinite(lr)) return fail(TP_EINVAL, "bad step or learning rate");
  if (!ws || ws_bytes < tp_mlp_train_workspace(ntensors, nslices))
    return fail(TP_EWORKSPACE, "training workspace too small");
  return mlp_train_step(params, m, v, step, lr, feat, target, ntensors, nslices, loss, grad, ws, S(stream));
}

size_t tp_mlp_proposal_workspace(const tp_tensor* A) {
  if (!A) return 0;
  return mlp_features_ws(A->n1, A->n2) + align_up(size_t(A->n2) * 17 * 4) + align_up(size_t(A->n2) * 4) + 2048;
}

int tp_mlp_proposal(const float* params, const tp_tensor* A, const float* phi, double alpha, double* w, void* ws,
                    size_t ws_bytes, void* stream) {
  if (int rc = check_a(A)) return rc;
  if (!params || !phi || !w) return fail(TP_EINVAL, "null pointer");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(TP_EINVAL, "alpha must lie in [0, 1]");
  if (!ws || ws_bytes < tp_mlp_proposal_workspace(A)) return fail(TP_EWORKSPACE, "proposal workspace too small");
  hipStream_t st = S(stream);
  Arena ar(ws, ws_bytes);
  void* fws = ar.take<char>(mlp_features_ws(A->n1, A->n2));
  float* feat = ar.take<float>(A->n2 * 17);
  float* logit = ar.take<float>(A->n2);
  if (!ar.ok()) return fail(TP_EWORKSPACE, "proposal workspace too small");
  if (int rc = mlp_features((const float*)A->data, A->n1, A->n2, A->n3, phi, feat, fws, st)) return rc;
  if (int rc = mlp_forward(params, feat, A->n2, logit, st)) return rc;
  return mlp_proposal(logit, A->n2, alpha, w, st);
}

}  // extern "C"

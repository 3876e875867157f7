// C ABI of the rank-predictor network (declared in include/hm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "api_util.h"
#include "mlp.h"

using namespace hm;

struct hm_mlp {
  hm::AllocRef alloc;       // the allocator of the context that made it
  float* master = nullptr;  // FP32 master weights (MLP_NPARAM)
  float* mom1 = nullptr;    // Adam moments
  float* mom2 = nullptr;
  float* grad = nullptr;
  void* work = nullptr;     // BF16 matrices + FP32 biases
  MlpWeights w{};
  int step = 0;
};

namespace {

// splitmix64 (Steele, Lea, Flood 2014) for a seeded initialisation
uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& s) { return ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

// He initialisation: N(0, 2 / fan_in) weights (Box-Muller), zero biases
std::vector<float> he_init(uint64_t seed) {
  std::vector<float> w(MLP_NPARAM, 0.0f);
  uint64_t s = seed;
  auto normal = [&]() {
    const double u1 = uniform01(s), u2 = uniform01(s);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  };
  for (int i = 0; i < MLP_H * MLP_IN; ++i) w[MLP_OFF_W1 + i] = (float)(normal() * std::sqrt(2.0 / MLP_IN));
  for (int i = 0; i < MLP_H * MLP_H; ++i) w[MLP_OFF_W2 + i] = (float)(normal() * std::sqrt(2.0 / MLP_H));
  for (int i = 0; i < MLP_H; ++i) w[MLP_OFF_W3 + i] = (float)(normal() * std::sqrt(2.0 / MLP_H));
  return w;
}

float bf16_round_host(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u = ((u + 0x7fffu + ((u >> 16) & 1u)) >> 16) << 16;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

}  // namespace

namespace hm {
MlpWeights hm_mlp_weights(const hm_mlp* n) { return n->w; }
}  // namespace hm

extern "C" {

hm_status hm_mlp_create(hm_ctx* ctx, const float* init, uint64_t seed, hm_mlp** out) {
  return guard([&] {
    if (!ctx || !out) return fail(HM_ERR_ARG, "hm_mlp_create: NULL argument");
    auto n = std::make_unique<hm_mlp>();
    const size_t pb = sizeof(float) * MLP_NPARAM;
    n->alloc = ctx->alloc;
    check(n->alloc->get(&n->master, pb), "allocate(mlp)");
    check(n->alloc->get(&n->mom1, pb), "allocate(mlp)");
    check(n->alloc->get(&n->mom2, pb), "allocate(mlp)");
    check(n->alloc->get(&n->grad, pb), "allocate(mlp)");
    const size_t wb = 2 * (MLP_H * MLP_IN + MLP_H * MLP_H + MLP_H) + 4 * (2 * MLP_H + 1) + 64;
    check(n->alloc->get(&n->work, wb), "allocate(mlp)");
    char* b = (char*)n->work;
    n->w.W1 = (uint16_t*)b;
    n->w.W2 = n->w.W1 + MLP_H * MLP_IN;
    n->w.w3 = n->w.W2 + MLP_H * MLP_H;
    n->w.b1 = (float*)(b + ((2 * (MLP_H * MLP_IN + MLP_H * MLP_H + MLP_H) + 15) & ~15));
    n->w.b2 = n->w.b1 + MLP_H;
    n->w.b3 = n->w.b2 + MLP_H;
    std::vector<float> w = init ? std::vector<float>(init, init + MLP_NPARAM) : he_init(seed);
    check(hipMemcpy(n->master, w.data(), pb, hipMemcpyHostToDevice), "mlp upload");
    check(hipMemset(n->mom1, 0, pb), "mlp zero");
    check(hipMemset(n->mom2, 0, pb), "mlp zero");
    check(mlp_publish(n->master, n->w, ctx->stream), "mlp publish");
    check(hipStreamSynchronize(ctx->stream), "mlp sync");
    *out = n.release();
    return HM_OK;
  });
}

void hm_mlp_free(hm_mlp* n) {
  if (!n) return;
  if (n->alloc) {
    n->alloc->put(n->master);
    n->alloc->put(n->mom1);
    n->alloc->put(n->mom2);
    n->alloc->put(n->grad);
    n->alloc->put(n->work);
  }
  delete n;
}

hm_status hm_mlp_get(hm_ctx* ctx, const hm_mlp* n, float* master, float* working) {
  return guard([&] {
    if (!ctx || !n) return fail(HM_ERR_ARG, "hm_mlp_get: NULL argument");
    check(hipStreamSynchronize(ctx->stream), "mlp sync");
    std::vector<float> w(MLP_NPARAM);
    check(hipMemcpy(w.data(), n->master, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost), "mlp read");
    if (master) std::memcpy(master, w.data(), sizeof(float) * MLP_NPARAM);
    if (working) {
      // the working copy is the BF16 rounding of the master weights (biases FP32)
      for (int i = 0; i < MLP_NPARAM; ++i) {
        const bool matrix = i < MLP_OFF_B1 || (i >= MLP_OFF_W2 && i < MLP_OFF_B2) || (i >= MLP_OFF_W3 && i < MLP_OFF_B3);
        working[i] = matrix ? bf16_round_host(w[i]) : w[i];
      }
    }
    return HM_OK;
  });
}

hm_status hm_mlp_predict(hm_ctx* ctx, const hm_mlp* n, const float* X, int64_t B, float* y) {
  return guard([&] {
    if (!ctx || !n || B < 0 || (B > 0 && (!X || !y))) return fail(HM_ERR_ARG, "hm_mlp_predict: invalid argument");
    check(mlp_forward(n->w, X, B, y, ctx->stream), "mlp forward");
    check(hipStreamSynchronize(ctx->stream), "mlp sync");
    return HM_OK;
  });
}

hm_status hm_mlp_gradient(hm_ctx* ctx, const hm_mlp* n, const float* X, const float* t, int64_t B, float* grad,
                          double* loss) {
  return guard([&] {
    if (!ctx || !n || B < 1 || !X || !t || !grad) return fail(HM_ERR_ARG, "hm_mlp_gradient: invalid argument");
    const int nblk = mlp_backward_blocks(B);
    float *partial = nullptr, *lb = nullptr;
    check(ctx->alloc->get(&partial, sizeof(float) * MLP_NPARAM * (size_t)nblk), "allocate(partial)");
    hipError_t e = ctx->alloc->get(&lb, sizeof(float) * nblk);
    if (e == hipSuccess) e = mlp_gradient(n->w, X, t, B, 1.0f / (float)B, partial, n->grad, lb, ctx->stream);
    std::vector<float> l(nblk);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipMemcpy(grad, n->grad, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(l.data(), lb, sizeof(float) * nblk, hipMemcpyDeviceToHost);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->alloc->put(partial);
    ctx->alloc->put(lb);
    check(e, "hm_mlp_gradient");
    if (loss) {
      double s = 0;
      for (float v : l) s += v;
      *loss = s / (double)B;
    }
    return HM_OK;
  });
}

hm_status hm_mlp_train(hm_ctx* ctx, hm_mlp* n, const float* X, const float* t, int64_t B, int32_t epochs,
                       int32_t batch, float lr, float* epoch_loss) {
  return guard([&] {
    if (!ctx || !n || B < 1 || !X || !t || epochs < 0 || batch < 1 || !(lr > 0))
      return fail(HM_ERR_ARG, "hm_mlp_train: invalid argument");
    const int64_t bs = std::min<int64_t>(batch, B);
    const int nblk = mlp_backward_blocks(bs);
    const int64_t nbatch = B / bs;  // full mini-batches of the (caller-shuffled) data
    float *partial = nullptr, *lb = nullptr;
    check(ctx->alloc->get(&partial, sizeof(float) * MLP_NPARAM * (size_t)nblk), "allocate(partial)");
    hipError_t e = ctx->alloc->get(&lb, sizeof(float) * nblk * (size_t)nbatch);
    std::vector<float> l((size_t)nblk * nbatch);
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
      for (int64_t q = 0; q < nbatch && e == hipSuccess; ++q) {
        e = mlp_gradient(n->w, X + q * bs * MLP_IN, t + q * bs, bs, 1.0f / (float)bs, partial, n->grad,
                         lb + q * nblk, ctx->stream);
        if (e == hipSuccess) e = mlp_adam(n->master, n->mom1, n->mom2, n->grad, lr, ++n->step, n->w, ctx->stream);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (e == hipSuccess) e = hipMemcpy(l.data(), lb, sizeof(float) * l.size(), hipMemcpyDeviceToHost);
      if (e == hipSuccess && epoch_loss) {
        double s = 0;
        for (float v : l) s += v;
        epoch_loss[ep] = (float)(s / (double)(nbatch * bs));
      }
    }
    (void)hipStreamSynchronize(ctx->stream);
    ctx->alloc->put(partial);
    ctx->alloc->put(lb);
    check(e, "hm_mlp_train");
    return HM_OK;
  });
}

}  // extern "C"

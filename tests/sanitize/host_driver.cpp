// Calls the host side of the C ABI on its validation and error paths,
// which need no GPU, so that a host-only build of the library with
// AddressSanitizer and UndefinedBehaviorSanitizer can check them.  Exit
// status 0 when every call returned the expected status.
#include <cstdint>
#include <cstdio>

#include "../../include/vflb.h"

static int fails = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("unexpected: %s\n", what);
    ++fails;
  }
}

int main() {
  vflb_sim* s = nullptr;
  expect(vflb_create(7, 8, 8, 1, VFLB_F32, nullptr, &s) == VFLB_EINVAL, "lattice");
  expect(vflb_last_error(nullptr)[0] != 0, "create error message");
  expect(vflb_create(VFLB_D2Q9, 8, 8, 1, 9, nullptr, &s) == VFLB_EINVAL, "storage");
  expect(vflb_create(VFLB_D2Q9, 0, 8, 1, VFLB_F32, nullptr, &s) == VFLB_EINVAL, "size");
  expect(vflb_create(VFLB_D3Q19, 16, 16, 16, VFLB_BF16S, nullptr, &s) == VFLB_EINVAL, "bf16 3d");
  expect(vflb_create(VFLB_D3Q19, 512, 512, 513, VFLB_F32, nullptr, &s) == VFLB_EINVAL, "3d size");
  expect(vflb_create_ex(VFLB_D2Q9, 8, 8, 1, VFLB_F32, 0, 2, nullptr, &s) == VFLB_EINVAL, "option");
  expect(vflb_create_ex(VFLB_D3Q19, 8, 8, 8, VFLB_F16S, 0, VFLB_OPT_INPLACE, nullptr, &s) ==
             VFLB_EINVAL, "in place 3d 16-bit");
  expect(vflb_copy_probe(reinterpret_cast<void*>(16), reinterpret_cast<void*>(32), 32, 4,
                         nullptr) == VFLB_EINVAL, "copy kind");
  expect(vflb_create_scheme(VFLB_D2Q9, 8, 8, 1, VFLB_F16S, VFLB_SCHEME_STRESS_DIVERGENCE, nullptr,
                            &s) == VFLB_EINVAL, "scheme 16-bit");
  expect(vflb_create(VFLB_D2Q9, 8, 8, 1, VFLB_F32, nullptr, nullptr) == VFLB_EINVAL, "out");
  expect(s == nullptr, "no handle after failures");
  // a valid lattice: created (a GPU is present) or refused at its stream
  vflb_status rc = vflb_create(VFLB_D2Q9, 8, 8, 1, VFLB_F32, nullptr, &s);
  expect(rc == VFLB_OK || rc == VFLB_EDEVICE, "valid create");
  if (rc == VFLB_OK) {
    size_t bytes[VFLB_NBUF];
    expect(vflb_query_buffers(s, bytes) == VFLB_OK, "query");
    vflb_params p{1.0, 1.0, 0.5, 0.01, 10.0, 0.0, 0.0};
    expect(vflb_set_params(s, &p) == VFLB_OK, "params");
    p.beta = 2.0;
    expect(vflb_set_params(s, &p) == VFLB_EINVAL, "bad beta");
    expect(vflb_step(s, 1) == VFLB_ESTATE, "step unbound");
    vflb_destroy(s);
  }
  // NULL handles
  expect(vflb_step(nullptr, 1) == VFLB_EINVAL, "step NULL");
  expect(vflb_set_params(nullptr, nullptr) == VFLB_EINVAL, "params NULL");
  double out[14];
  expect(vflb_reduce(nullptr, out) == VFLB_EINVAL, "reduce NULL");
  expect(vflb_reduce_noalloc(nullptr, out) == VFLB_EINVAL, "reduce_noalloc NULL");
  vflb_destroy(nullptr);
  // batches
  vflb_batch* b = nullptr;
  int dims[6] = {64, 64, 1, 32, 16, 1};
  expect(vflb_batch_create(VFLB_D3Q19, 2, dims, VFLB_F32, nullptr, &b) == VFLB_EINVAL, "batch 3d");
  expect(vflb_batch_create(VFLB_D2Q9, 0, dims, VFLB_F32, nullptr, &b) == VFLB_EINVAL, "batch n");
  int bad[6] = {64, 64, 1, 0, 16, 1};
  expect(vflb_batch_create(VFLB_D2Q9, 2, bad, VFLB_F32, nullptr, &b) == VFLB_EINVAL, "batch dims");
  expect(vflb_batch_last_error(nullptr)[0] != 0, "batch error message");
  expect(b == nullptr, "no batch after failures");
  vflb_batch_destroy(nullptr);
  // networks
  vflb_mlp* m = nullptr;
  vflb_mlp_cfg c{5, 128, 256, 3, 5, 1024, 1.5};
  vflb_mlp_cfg w = c;
  w.width = 100;
  expect(vflb_mlp_create(&w, nullptr, &m) == VFLB_EINVAL, "mlp width");
  w = c;
  w.n_freq = 20;
  expect(vflb_mlp_create(&w, nullptr, &m) == VFLB_EINVAL, "mlp freq");
  w = c;
  w.max_batch = 100;
  expect(vflb_mlp_create(&w, nullptr, &m) == VFLB_EINVAL, "mlp batch");
  expect(vflb_mlp_create(&c, nullptr, &m) == VFLB_OK, "mlp create");
  size_t mb[VFLB_MLP_NBUF];
  expect(vflb_mlp_query_buffers(m, mb) == VFLB_OK && mb[0] > 0 && mb[1] > 0, "mlp buffers");
  expect(vflb_mlp_param_count(m) == 128 * 5 + 198661, "mlp params");
  double loss = 0.0;
  expect(vflb_mlp_train(m, nullptr, nullptr, 10, 10, 1, 1e-3f, 1, 0, nullptr) == VFLB_ESTATE,
         "train unbound");
  expect(vflb_mlp_train_step(m, nullptr, nullptr, 10, 1e-3f, &loss) == VFLB_ESTATE,
         "train step unbound");
  vflb_mlp_destroy(m);
  // copy probe argument checks
  expect(vflb_stream_copy(reinterpret_cast<void*>(16), reinterpret_cast<void*>(32), 17, nullptr) ==
             VFLB_EINVAL, "copy size");
  std::printf("host driver: %d unexpected\n", fails);
  return fails ? 1 : 0;
}

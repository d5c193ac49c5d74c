// Sanitizer driver for libmpm's host-only logic: the binomial schedule
// (mpm_revolve_steps / mpm_revolve_split) over a range of lengths and slot
// counts, error strings, and the argument checks that return before any
// HIP call (mpm_init, mpm_step_forward_noalloc).  Linked into an executable
// built with host-side address and undefined-behaviour sanitizers by
// tests/test_sanitizers.py (no GPU is touched).
#include <cstdio>
#include <cstring>

#include "../../include/mpm.h"

int main() {
  int bad = 0;
  for (int64_t L = 0; L <= 300; ++L)
    for (int s = 0; s <= 12; ++s) {
      const int64_t c = mpm_revolve_steps(L, s);
      if (c < 0 && L > 0 && s > 0) ++bad;
      if (L > 1 && s > 0) {
        const int64_t m = mpm_revolve_split(L, s);
        if (m < 1 || m >= L) ++bad;
      }
    }
  if (mpm_revolve_steps(-1, 2) >= 0) ++bad;
  for (int code = -8; code <= 0; ++code)
    if (!mpm_strerror(code) || !std::strlen(mpm_strerror(code))) ++bad;
  mpm_ctx *ctx = nullptr;
  mpm_scene sc;
  std::memset(&sc, 0, sizeof sc);
  sc.dim = 2;
  sc.n_grid = 16;
  sc.n_particles = 4;
  sc.wall = 3;
  sc.dt = 1e-4f;
  sc.E = 10.0f;
  sc.nu = 0.3f;
  sc.rho = 1.0f;
  sc.V0 = 1e-3f;
  if (mpm_init(nullptr, &sc, 1, nullptr, nullptr, nullptr) != MPM_ERR_ARG) ++bad;
  if (mpm_init(&ctx, nullptr, 1, nullptr, nullptr, nullptr) != MPM_ERR_ARG) ++bad;
  mpm_scene s2 = sc;
  s2.dim = 5;
  if (mpm_init(&ctx, &s2, 1, nullptr, nullptr, nullptr) != MPM_ERR_ARG) ++bad;
  s2 = sc;
  s2.nu = 0.5f;
  if (mpm_init(&ctx, &s2, 1, nullptr, nullptr, nullptr) != MPM_ERR_ARG) ++bad;
  mpm_opts o;
  std::memset(&o, 0, sizeof o);
  o.fusion = 3;
  if (mpm_init(&ctx, &sc, 1, nullptr, nullptr, &o) != MPM_ERR_ARG) ++bad;
  if (ctx != nullptr) ++bad;
  mpm_state st = {nullptr, nullptr, nullptr, nullptr};
  uint32_t err = 0;
  if (mpm_step_forward_noalloc(nullptr, nullptr, &st, nullptr, &st, &err, nullptr) !=
      MPM_ERR_ARG)
    ++bad;
  s2 = sc;
  s2.n_grid = 1024;  // 1024^2 nodes: beyond the allocation-free region
  if (mpm_step_forward_noalloc(&s2, nullptr, &st, nullptr, &st, &err, nullptr) != MPM_ERR_ARG)
    ++bad;
  if (mpm_set_horizons(nullptr, nullptr) != MPM_ERR_ARG) ++bad;
  std::printf("host sanitizer run: %d problems\n", bad);
  return bad ? 1 : 0;
}

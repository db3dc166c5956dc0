// Checkpoint schedule for the reverse pass through a chain of n stout levels
// U_0 -> U_1 -> ... -> U_n (host-only code).
//
// The adjoint of level l maps the gradient from U_l to U_{l-1} and needs
// U_{l-1}; it runs for l = n, n-1, ..., 1.  U_0 (the thin links) is always
// available; the forward pass that builds U_n for the solver visits every
// level once, and may keep up to s of them in checkpoint slots at no extra
// cost.  Any other level the reverse pass needs is recomputed by smearing
// forward from an available one (one pass per level), either into a slot
// (a new checkpoint) or into a transient buffer that serves one adjoint.
//
// The schedule minimises the number of recomputed passes, by dynamic
// programming over two costs (segment [a, b] of length l = b - a, U_a
// available, the adjoints of levels b .. a+1 to run, k free slots):
//   F(l, k): U_a was reached in the reverse pass, so reaching U_{a+m}
//            costs m passes:
//            F(1, k) = 0,  F(l, 0) = l(l-1)/2  (each level from U_a),
//            F(l, k) = min_m [ m + F(l-m, k-1) + F(m, k) ]
//            (advance m levels into a slot, serve the right part with one
//            slot fewer, free the slot, serve the left part);
//   G(l, k): the same on the forward pass's path, where storing U_{a+m} is
//            free:  G(1, k) = 0,  G(l, 0) = l(l-1)/2,
//            G(l, k) = min_m [ G(l-m, k-1) + F(m, k) ].
// The reverse pass costs G(n, s) smearing passes: 0 with s >= n - 1 slots
// (store every level), n(n-1)/2 with none.  This is the binomial
// checkpointing idea (Griewank's treeverse) specialised to a forward sweep
// that is already paid for.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace lgt {

constexpr int kMaxStoutLevels = 256;

class StoutSchedule {
 public:
  StoutSchedule() = default;
  StoutSchedule(int n, int s) : n_(n), s_(std::max(0, std::min(s, n - 1))) {
    const int L = n_ + 1, K = s_ + 1;
    F_.assign((size_t)L * K, 0);
    Fm_.assign((size_t)L * K, 0);
    G_.assign((size_t)L * K, 0);
    Gm_.assign((size_t)L * K, 0);
    for (int l = 1; l <= n_; ++l) {
      for (int k = 0; k <= s_; ++k) {
        int64_t f, g;
        int fm = 0, gm = 0;
        if (l == 1) {
          f = g = 0;
        } else if (k == 0) {
          f = g = (int64_t)l * (l - 1) / 2;
        } else {
          f = g = INT64_MAX;
          for (int m = 1; m < l; ++m) {
            const int64_t cf = m + at(F_, l - m, k - 1) + at(F_, m, k);
            if (cf < f) f = cf, fm = m;
            const int64_t cg = at(G_, l - m, k - 1) + at(F_, m, k);
            if (cg < g) g = cg, gm = m;
          }
        }
        set(F_, l, k, f);
        set(G_, l, k, g);
        Fm_[(size_t)l * K + k] = fm;
        Gm_[(size_t)l * K + k] = gm;
      }
    }
  }
  int levels() const { return n_; }
  int slots() const { return s_; }
  // smearing passes of the reverse pass beyond the forward sweep
  int64_t cost() const { return n_ >= 1 ? at(G_, n_, s_) : 0; }
  int64_t cost_F(int l, int k) const { return at(F_, l, std::min(k, s_)); }
  // split of a reverse-pass segment (F) / forward-path segment (G); 0 = none
  int split_F(int l, int k) const { return Fm_[(size_t)l * (s_ + 1) + std::min(k, s_)]; }
  int split_G(int l, int k) const { return Gm_[(size_t)l * (s_ + 1) + std::min(k, s_)]; }
  // levels the forward sweep stores, in increasing order (slot i holds the i-th)
  std::vector<int> forward_checkpoints() const {
    std::vector<int> p;
    int a = 0, k = s_;
    while (n_ - a > 1 && k > 0) {
      const int m = split_G(n_ - a, k);
      a += m;
      p.push_back(a);
      --k;
    }
    return p;
  }

 private:
  int64_t at(const std::vector<int64_t>& t, int l, int k) const { return t[(size_t)l * (s_ + 1) + k]; }
  void set(std::vector<int64_t>& t, int l, int k, int64_t v) { t[(size_t)l * (s_ + 1) + k] = v; }
  int n_ = 0, s_ = 0;
  std::vector<int64_t> F_, G_;
  std::vector<int> Fm_, Gm_;
};

}  // namespace lgt

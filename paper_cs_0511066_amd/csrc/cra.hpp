// Early-terminated Chinese remaindering of one matrix run in rounds (the CRA
// loop of Section 2.1, Alg. 2.1, with the run length of Lemma 2.1(iv)), as
// the batched and serving loops drive it: each round draws the matrix's next
// primes, their residues come back from the device, and the host folds them
// in draw order into the symmetric-range Garner reconstruction, stopping at
// k unchanged reconstructions (early termination) or at the deterministic
// bound prod p >= 2H.
#pragma once
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "bigint.hpp"
#include "host_numerics.hpp"

namespace dethost {

struct CraJob {
  Bounds bd;
  int n = 0;
  bool certify = false;
  double log2_l = 22.0;
  std::unique_ptr<PrimeSampler> samp;
  CrtState crt;
  int64_t kET = 0;     // run length of Lemma 2.1(iv)
  int64_t cert = 0;    // primes that reach the deterministic bound 2H
  int rounds = 0;
  bool done = false;
  bool early = false;  // stopped by early termination
  std::vector<uint32_t> ps;   // this round's primes, in draw order
  int64_t res0 = 0;           // where their residues go in the round's array

  // Primes drawn from (2^(bits-1), 2^bits) by the stream seeded with `seed`.
  void init(const Bounds& b, int order, uint64_t seed, int bits, double log2_inv_eps, bool cert_mode) {
    bd = b;
    n = order;
    certify = cert_mode;
    log2_l = (double)(bits - 1);
    samp.reset(new PrimeSampler(splitmix64(seed), bits));
    const double logl_H = std::max(1.0, bd.log2_h / log2_l);
    kET = et_run_length(log2_inv_eps, prime_set_size(bits), logl_H);
    if (kET < 0) kET = INT64_MAX;
    cert = (int64_t)ceil((bd.log2_h + 2.0) / log2_l) + 1;
    rounds = 0;
    done = false;
  }

  // Primes of the next round.  First round: enough for the expected size of
  // |det| of a dense matrix with independent entries (log2 H less n log2(e)/2,
  // plus 32 bits) and the run length; certify: the deterministic bound.
  // Later rounds: what the bound still needs, capped at twice the run length.
  int64_t next_count() const {
    const int64_t k = std::min<int64_t>(kET, 64);
    int64_t want;
    if (rounds == 0) {
      const double est = std::max(1.0, bd.log2_h - 0.5 * n * 1.4426950408889634 + 32.0);
      want = certify ? cert : std::min<int64_t>(cert, (int64_t)ceil(est / log2_l) + k + 1);
    } else {
      const double need = (bd.log2_h + 2.0 - (double)(crt.M.bit_length() - 1)) / log2_l;
      want = std::min<int64_t>(std::max<int64_t>((int64_t)ceil(need) + 1, 4), 4096);
      if (!certify) want = std::min<int64_t>(want, std::max<int64_t>(2 * k, 8));
    }
    return std::max<int64_t>(want, 1);
  }

  void draw(int64_t count, int64_t at) {
    ps.resize(count);
    for (auto& q : ps) q = samp->next();
    res0 = at;
  }

  // Folds this round's residues (res[res0 + i] for ps[i]) in draw order.
  bool absorb(const uint32_t* res) {
    for (size_t k = 0; k < ps.size() && !done; k++) {
      crt.add(ps[k], res[res0 + k]);
      if ((double)(crt.M.bit_length() - 1) >= bd.log2_h + 2.0) done = true;
      else if (!certify && crt.same >= kET) {
        done = true;
        early = true;
      }
    }
    ps.clear();
    rounds++;
    return done;
  }
};

}  // namespace dethost

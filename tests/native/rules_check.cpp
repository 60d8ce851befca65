// Host check of the FIFO rules the kernels use (prune_rules.h): seeded random
// write/read traffic on FIFOs of every rate, delay and C within small bounds,
// each write and read allowed only when the blocking rules allow it.  Tokens
// are numbered and stored at the slots the Fig. 6 rule gives (with the
// copy-back of unaligned delays), and every read must return the next tokens
// in stream order.  The occupancy stays within Eq. 2 (fifo_state_ok), the
// counters only grow, and every access stays inside the buffer.  The checks
// that PRUNE_DEBUG builds of the bookkeeping kernels run after each counter
// update (fifo_counters_ok, fifo_advance_ok) hold on every state of that
// traffic, with variable token counts per block, and fail on planted
// mistakes: a read past the delay and the writes, a write past the buffer,
// a counter going back, a block with more than r tokens.  Also checks the
// configuration mapping's masks against the bank they address.  Built with
// ASan/UBSan; prints "ok <cases> <accesses> <planted>" or the first failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "prune_rules.h"

using namespace prune;

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next(uint32_t n) {
  rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
  return (uint32_t)(rng % n);
}

#define CHECK(c, ...) do { if (!(c)) { std::printf(__VA_ARGS__); std::printf("\n"); return 1; } } while (0)

int main() {
  uint64_t cases = 0, accesses = 0;
  for (uint32_t r = 1; r <= 6; ++r)
    for (uint32_t C = 1; C <= 4; ++C)
      for (uint32_t Q = 0; Q <= 3 * r * C; ++Q) {
        if (Q % r && (Q >= r * C || (Q < r && Q + r > r * C))) continue;   // rejected at finalize
        const uint64_t cap = fifo_capacity(r, Q, C);
        std::vector<int64_t> buf(cap, -1);
        // delay tokens are stream tokens 0..Q-1 (value -2-k), data tokens follow
        for (uint64_t k = 0; k < Q; ++k) buf[k] = -2 - (int64_t)k;
        uint64_t writes = 0, reads = 0, next_tok = 0, next_read_tok = 0;
        // token counters of a variable-rate FIFO on the same block traffic:
        // block j carries cnt[j] in 1..r tokens
        std::vector<uint32_t> cnt;
        uint64_t tw = 0, tr = 0;
        for (int step = 0; step < 400; ++step) {
          const int64_t inflight = (int64_t)writes - (int64_t)reads;
          CHECK(fifo_state_ok(r, Q, C, inflight), "state r=%u Q=%u C=%u inflight=%lld", r, Q, C, (long long)inflight);
          CHECK(fifo_counters_ok(r, Q, C, writes, reads, tw, tr), "counters r=%u Q=%u C=%u w=%llu rd=%llu", r, Q,
                C, (unsigned long long)writes, (unsigned long long)reads);
          const bool w = next(2), can_w = fifo_can_write(r, Q, C, inflight), can_r = fifo_can_read(r, Q, C, inflight);
          CHECK(can_w || can_r, "stuck r=%u Q=%u C=%u", r, Q, C);
          if ((w && can_w) || !can_r) {
            const uint64_t s = fifo_write_slot(r, Q, C, writes);
            CHECK(s + r <= cap, "write out of buffer r=%u Q=%u C=%u j=%llu", r, Q, C, (unsigned long long)writes);
            for (uint32_t k = 0; k < r; ++k) buf[s + k] = (int64_t)(next_tok + k);
            if (Q % r && s + r > (uint64_t)r * C)
              for (uint64_t k = (uint64_t)r * C; k < s + r; ++k) buf[k - (uint64_t)r * C] = buf[k];
            next_tok += r;
            cnt.push_back(1 + next(r));
            CHECK(fifo_advance_ok(r, writes, tw, writes + 1, tw + cnt.back()), "write advance");
            tw += cnt.back();
            ++writes;
          } else {
            const uint64_t s = fifo_read_slot(r, Q, C, reads);
            CHECK(s + r <= cap, "read out of buffer r=%u Q=%u C=%u i=%llu", r, Q, C, (unsigned long long)reads);
            for (uint32_t k = 0; k < r; ++k) {
              const uint64_t t = next_read_tok + k;   // stream position
              const int64_t want = t < Q ? -2 - (int64_t)t : (int64_t)(t - Q);
              CHECK(buf[s + k] == want, "order r=%u Q=%u C=%u read %llu slot %llu: %lld != %lld", r, Q, C,
                    (unsigned long long)reads, (unsigned long long)(s + k), (long long)buf[s + k], (long long)want);
            }
            next_read_tok += r;
            // the first Q/r blocks read are the delay's (r tokens each, and
            // an unaligned delay's partial block is read with the first data)
            const uint64_t got = reads < Q / r ? r : cnt[reads - Q / r];
            CHECK(fifo_advance_ok(r, reads, tr, reads + 1, tr + got), "read advance");
            tr += got;
            ++reads;
          }
          ++accesses;
        }
        ++cases;
      }
  // planted mistakes: every state past the buffer or before the delay, a
  // counter going back, more than r tokens in a block
  uint64_t planted = 0;
  for (uint32_t r = 1; r <= 6; ++r)
    for (uint32_t C = 1; C <= 4; ++C)
      for (uint32_t Q = 0; Q <= 3 * r * C; ++Q) {
        if (Q % r && (Q >= r * C || (Q < r && Q + r > r * C))) continue;
        const uint64_t cap = fifo_capacity(r, Q, C);
        const uint64_t base = 100;   // reads so far
        for (int64_t d = -(int64_t)(Q / r) - 3; d <= (int64_t)(cap / r) + 3; ++d) {
          const uint64_t w = base + d, rd = base;
          // whole blocks of r tokens: the slots held are Q + d r
          const int64_t held = (int64_t)Q + d * (int64_t)r;
          const bool fits = d >= -(int64_t)(Q / r) && held >= 0 && (uint64_t)held <= cap;
          const bool ok = fifo_counters_ok(r, Q, C, w, rd, w * r, rd * r);
          CHECK(ok == fits, "occupancy r=%u Q=%u C=%u d=%lld: ok=%d fits=%d", r, Q, C, (long long)d, ok, fits);
          if (!fits) ++planted;
          // tokens beyond r per block written or read
          if (fits && w > 0) {
            CHECK(!fifo_counters_ok(r, Q, C, w, rd, w * r + 1, rd * r), "tokens past r per write block r=%u Q=%u C=%u d=%lld", r, Q, C, (long long)d);
            CHECK(!fifo_counters_ok(r, Q, C, w, rd, w * r, rd * r + 1), "tokens past r per read block");
            planted += 2;
          }
        }
        CHECK(!fifo_advance_ok(r, 5, 5, 4, 5), "access counter going back");
        CHECK(!fifo_advance_ok(r, 5, 5, 5, 4), "token counter going back");
        CHECK(!fifo_advance_ok(r, 5, 5, 6, 5 + r + 1), "more than r tokens in one block");
        CHECK(!fifo_advance_ok(r, 5, 5, 5, 6), "tokens without an access");
        CHECK(fifo_advance_ok(r, 5, 5, 8, 5 + 3 * r), "three full blocks");
        planted += 4;
      }
  // configuration mapping: the mask addresses only the bank's branches
  for (uint32_t mode = 0; mode < 3; ++mode)
    for (int t = 0; t < 20000; ++t) {
      // records the configuration actor accepts: K <= Kmax (prefix), K < 2^Kmax (mask)
      const uint32_t Kmax = 1 + next(10);
      prune_side_info s{mode == PRUNE_CONFIG_MASK ? next(1u << Kmax) : next(Kmax + 1), 1 + next(1000),
                        next(4), next(3)};
      const prune_ctrl_token k = config_map(mode, Kmax, s);
      CHECK(k.rate == s.n, "rate");
      if (mode == PRUNE_CONFIG_ROUTE) {
        CHECK(k.mask == (1u << s.route), "route mask");
      } else {
        const uint32_t sh = s.bank * Kmax;
        const uint64_t bank_bits = ((1ull << Kmax) - 1ull) << sh;
        CHECK(sh >= 32 || (k.mask & ~bank_bits) == 0, "mask outside its bank");
        for (uint32_t e = 1; e <= 32; ++e)
          CHECK(decode_bit(k.mask, e) == ((k.mask >> (e - 1)) & 1u), "decode");
      }
    }
  std::printf("ok %llu %llu %llu\n", (unsigned long long)cases, (unsigned long long)accesses,
              (unsigned long long)planted);
  return 0;
}

// Host-only checks of the serving runtime's scheduling logic on the fake
// device (fake_device.cpp): per-stream order and carries, the HBM budget and
// no head-of-line blocking, cancel, close while busy, export / import,
// allocation and launch failures, and many threads at once (run under
// ThreadSanitizer by tests/test_serve_host.py).
//
// TEST INFRASTRUCTURE ONLY. Prints one line per check; exit status 0 when all
// pass.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <random>
#include <thread>
#include <vector>

#include "rfi.h"

extern "C" void fake_fail_alloc_in(int k);
extern "C" void fake_fail_launch_in(int k);
extern "C" void fake_set_work_us(int us);
extern "C" int fake_errors();

static int g_fail = 0;
#define CHECK(c)                                                                   \
  do {                                                                             \
    if (!(c)) {                                                                    \
      std::printf("FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #c, rfi_last_error()); \
      std::fflush(stdout);                                                         \
      ++g_fail;                                                                    \
      return;                                                                      \
    }                                                                              \
  } while (0)

namespace {

constexpr int NB = 4, NC = 8, STRIDE = 16;

// A block's bytes (host memory stands in for device memory on the fake).
struct Block {
  std::vector<std::vector<uint8_t>> beams;
  rfi_block blk{};
  Block(int64_t nsamp, uint32_t seed) {
    std::mt19937 g(seed);
    beams.resize(NB);
    blk.nbeam = NB;
    blk.nchan = NC;
    blk.nsamp = nsamp;
    blk.row_stride = STRIDE;
    for (int b = 0; b < NB; ++b) {
      beams[b].resize((size_t)(nsamp > 0 ? nsamp : 1) * STRIDE);
      for (auto& v : beams[b]) v = (uint8_t)(g() & 255);
      blk.beam[b] = beams[b].data();
    }
  }
};

// The expected cells of one stream's blocks (the carry arithmetic restated).
struct Expect {
  int L;
  int64_t c = 0;         // carry samples
  int nclipped = 0;      // earlier blocks with cells
  struct One {
    int nsub, carried, seq;
    int64_t t_full, carry_after;
  };
  One next(int64_t n) {
    One o{0, 0, -1, 0, 0};
    int64_t t = 0;
    bool open = false;
    if (c > 0) {
      if (n >= L - c) {
        o.carried = 1;
        t = L - c;
      } else {
        open = true;
        c += n;
      }
    }
    o.t_full = t;
    if (!open) {
      const int64_t full = (n - t) / L;
      o.nsub = o.carried + (int)full;
      c = n - t - full * L;
    }
    o.carry_after = c;
    if (o.nsub > 0) o.seq = nclipped++;
    return o;
  }
};

rfi_session* make_session(int slots, int64_t budget) {
  rfi_session_config sc{0, slots, budget, nullptr};
  rfi_session* s = nullptr;
  if (rfi_session_create(&sc, &s) != RFI_OK) return nullptr;
  return s;
}

int open_stream(rfi_session* s, int L) {
  rfi_stream_config c{NB, NC, L, 32, 12, 50, 3.0, nullptr, 0, 0, 1.0};
  int32_t id = -1;
  if (rfi_stream_open(s, &c, &id) != RFI_OK) return -1;
  return id;
}

// Checks one finished block against the expectation (and releases it).
bool check_result(rfi_session* s, const rfi_result& r, const Block& b, const Expect::One& e,
                  int L) {
  if (r.status != RFI_OK || r.nsub != e.nsub || r.carried != e.carried ||
      r.carry_samples != e.carry_after) {
    std::printf("  block %llu: status %d nsub %d/%d carried %d/%d carry %lld/%lld\n",
                (unsigned long long)r.ticket, r.status, r.nsub, e.nsub, r.carried, e.carried,
                (long long)r.carry_samples, (long long)e.carry_after);
    return false;
  }
  if (e.nsub > 0 && r.flag.iterations != e.seq) {
    std::printf("  block %llu: clip sequence %d, expected %d\n", (unsigned long long)r.ticket,
                r.flag.iterations, e.seq);
    return false;
  }
  const size_t n = (size_t)e.nsub * NC;
  std::vector<double> stat(n + 1);
  std::vector<uint8_t> mask(n + 1), cs(n + 1);
  if (rfi_result_copy(s, r.ticket, stat.data(), cs.data(), mask.data()) != RFI_OK) return false;
  for (int k = 0; k < e.nsub; ++k)
    for (int j = 0; j < NC; ++j) {
      double want;
      if (k < e.carried)
        want = 100000.0 + L;
      else
        want = b.beams[0][(size_t)(e.t_full + (int64_t)(k - e.carried) * L) * STRIDE + j];
      const double got = stat[(size_t)k * NC + j];
      if (got != want || mask[(size_t)k * NC + j] != (got > 200.0)) {
        std::printf("  block %llu cell (%d, %d): %g, expected %g\n",
                    (unsigned long long)r.ticket, k, j, got, want);
        return false;
      }
    }
  return rfi_result_release(s, r.ticket) == RFI_OK;
}

// ---------------------------------------------------------------------------
void order_and_carries() {
  fake_set_work_us(300);
  rfi_session* s = make_session(3, 0);
  CHECK(s);
  const int Ls[3] = {16, 5, 32};
  int ids[3];
  Expect ex[3] = {{16}, {5}, {32}};
  for (int i = 0; i < 3; ++i) CHECK((ids[i] = open_stream(s, Ls[i])) > 0);
  const int64_t sizes[] = {40, 3, 16, 0, 17, 64, 1, 2, 31, 33, 8, 100};
  std::vector<std::unique_ptr<Block>> blocks;
  std::vector<uint64_t> tickets;
  std::vector<Expect::One> exp;
  std::vector<int> sid;
  uint32_t seed = 1;
  for (int64_t n : sizes)
    for (int i = 0; i < 3; ++i) {
      blocks.emplace_back(new Block(n, seed++));
      uint64_t t = 0;
      CHECK(rfi_submit(s, ids[i], &blocks.back()->blk, seed, &t) == RFI_OK);
      tickets.push_back(t);
      exp.push_back(ex[i].next(n));
      sid.push_back(i);
    }
  for (size_t k = 0; k < tickets.size(); ++k) {
    rfi_result r{};
    CHECK(rfi_wait(s, tickets[k], -1, &r) == RFI_OK);
    CHECK(r.user_tag == (uint64_t)(k + 2));
    CHECK(check_result(s, r, *blocks[k], exp[k], Ls[sid[k]]));
  }
  // (each clip saw the stream state its predecessor left: sequence checked above)
  rfi_session_destroy(s);
  CHECK(fake_errors() == 0);
  std::printf("ok order_and_carries\n");
}

// Sub-intervals past the int32 bound: the carry is summed by the long route
// (int64 records, counts after them), opened, extended, completed and opened
// again; an ordinary stream runs beside it.
void long_carries() {
  fake_set_work_us(50);
  rfi_session* s = make_session(2, 0);
  CHECK(s);
  const int Ls[2] = {RFI_MAX_COUNT + 7, 24};
  int ids[2];
  Expect ex[2] = {{Ls[0]}, {Ls[1]}};
  for (int i = 0; i < 2; ++i) CHECK((ids[i] = open_stream(s, Ls[i])) > 0);
  const int64_t sizes[2][5] = {{40000, 20000, 8000, 2, 70000}, {50, 3, 24, 100, 7}};
  std::vector<std::unique_ptr<Block>> blocks;
  std::vector<uint64_t> tickets;
  std::vector<Expect::One> exp;
  std::vector<int> sid;
  uint32_t seed = 900;
  for (int k = 0; k < 5; ++k)
    for (int i = 0; i < 2; ++i) {
      blocks.emplace_back(new Block(sizes[i][k], seed++));
      uint64_t t = 0;
      CHECK(rfi_submit(s, ids[i], &blocks.back()->blk, seed, &t) == RFI_OK);
      tickets.push_back(t);
      exp.push_back(ex[i].next(sizes[i][k]));
      sid.push_back(i);
    }
  for (size_t k = 0; k < tickets.size(); ++k) {
    rfi_result r{};
    CHECK(rfi_wait(s, tickets[k], -1, &r) == RFI_OK);
    CHECK(check_result(s, r, *blocks[k], exp[k], Ls[sid[k]]));
  }
  // one past the long bound is refused
  rfi_stream_config c{NB, NC, RFI_MAX_COUNT_LONG + 1, 32, 12, 50, 3.0, nullptr, 0, 0, 1.0};
  int32_t id = -1;
  CHECK(rfi_stream_open(s, &c, &id) == RFI_E_INVALID);
  rfi_session_destroy(s);
  CHECK(fake_errors() == 0);
  std::printf("ok long_carries\n");
}

void budget_and_no_head_of_line() {
  fake_set_work_us(3000);
  const int64_t big = (int64_t)NB * 2048 * STRIDE, small = (int64_t)NB * 256 * STRIDE;
  // the budget holds one big block and one small one, not two big ones
  rfi_session* s = make_session(4, big + small + 64 * 1024);
  CHECK(s);
  const int a = open_stream(s, 64), b = open_stream(s, 64);
  CHECK(a > 0 && b > 0);
  Block A1(2048, 1), A2(2048, 2), B1(256, 3), huge(2048 * 3, 4);
  uint64_t ta1, ta2, tb1, th;
  CHECK(rfi_submit(s, a, &huge.blk, 0, &th) == RFI_E_BUDGET);
  CHECK(rfi_submit(s, a, &A1.blk, 0, &ta1) == RFI_OK);
  CHECK(rfi_submit(s, a, &A2.blk, 0, &ta2) == RFI_OK);
  CHECK(rfi_submit(s, b, &B1.blk, 0, &tb1) == RFI_OK);
  rfi_result r1{}, r2{}, r3{};
  CHECK(rfi_wait(s, ta1, -1, &r1) == RFI_OK && r1.status == RFI_OK);
  CHECK(rfi_wait(s, ta2, -1, &r2) == RFI_OK && r2.status == RFI_OK);
  CHECK(rfi_wait(s, tb1, -1, &r3) == RFI_OK && r3.status == RFI_OK);
  // A2 could not start before A1 finished (budget); B1 passed A2 meanwhile
  CHECK(r2.t_admit_us >= r1.t_done_us);
  CHECK(r3.t_admit_us < r2.t_admit_us);
  CHECK(r3.t_admit_us < r1.t_done_us);
  for (uint64_t t : {ta1, ta2, tb1}) CHECK(rfi_result_release(s, t) == RFI_OK);
  rfi_session_destroy(s);
  std::printf("ok budget_and_no_head_of_line\n");
}

void cancel_and_close() {
  fake_set_work_us(50000);
  rfi_session* s = make_session(1, 0);
  CHECK(s);
  const int a = open_stream(s, 16);
  CHECK(a > 0);
  Block X1(64, 1), X2(64, 2), X3(64, 3);
  uint64_t t1, t2, t3;
  CHECK(rfi_submit(s, a, &X1.blk, 0, &t1) == RFI_OK);
  CHECK(rfi_submit(s, a, &X2.blk, 0, &t2) == RFI_OK);
  rfi_result r{};
  // X1 runs (one slot; admitted within microseconds, its work takes 100 ms),
  // X2 waits: X2 can be cancelled, X1 cannot
  std::this_thread::sleep_for(std::chrono::milliseconds(10));
  CHECK(rfi_cancel(s, t1) == RFI_E_NOT_READY);
  CHECK(rfi_cancel(s, t2) == RFI_OK);
  CHECK(rfi_wait(s, t2, -1, &r) == RFI_OK && r.status == RFI_E_CANCELLED);
  CHECK(rfi_cancel(s, t2) == RFI_E_NOT_READY);
  CHECK(rfi_wait(s, t1, 0, &r) == RFI_E_TIMEOUT);
  // close while busy: returns once the stream's work is done
  CHECK(rfi_submit(s, a, &X3.blk, 0, &t3) == RFI_OK);
  std::atomic<bool> closed{false};
  std::thread th([&] {
    rfi_stream_close(s, a);
    closed = true;
  });
  CHECK(rfi_wait(s, t3, -1, &r) == RFI_OK && r.status == RFI_OK);
  th.join();
  CHECK(closed);
  CHECK(rfi_poll(s, t1, &r) == RFI_OK && r.status == RFI_OK);
  uint64_t t4;
  CHECK(rfi_submit(s, a, &X1.blk, 0, &t4) == RFI_E_INVALID);   // closed stream
  for (uint64_t t : {t1, t2, t3}) CHECK(rfi_result_release(s, t) == RFI_OK);
  rfi_session_destroy(s);
  std::printf("ok cancel_and_close\n");
}

void export_import() {
  fake_set_work_us(100);
  rfi_session* s = make_session(2, 0);
  CHECK(s);
  const int a = open_stream(s, 16);
  Expect ex{16};
  Block B1(40, 9);
  uint64_t t;
  CHECK(rfi_submit(s, a, &B1.blk, 0, &t) == RFI_OK);
  rfi_result r{};
  CHECK(rfi_wait(s, t, -1, &r) == RFI_OK);
  CHECK(check_result(s, r, B1, ex.next(40), 16));
  size_t nb = 0;
  CHECK(rfi_stream_export(s, a, nullptr, &nb) == RFI_OK && nb > 0);
  std::vector<char> buf(nb);
  CHECK(rfi_stream_export(s, a, buf.data(), &nb) == RFI_OK);
  const int b = open_stream(s, 16);
  CHECK(rfi_stream_import(s, b, buf.data(), nb) == RFI_OK);
  Block B2(30, 10);
  CHECK(rfi_submit(s, b, &B2.blk, 0, &t) == RFI_OK);
  CHECK(rfi_wait(s, t, -1, &r) == RFI_OK);
  CHECK(check_result(s, r, B2, ex.next(30), 16));   // resumes the carry and the sequence
  rfi_session_destroy(s);
  std::printf("ok export_import\n");
}

void allocation_failure() {
  fake_set_work_us(100);
  rfi_session* s = make_session(1, 0);
  CHECK(s);
  const int a = open_stream(s, 16);
  Expect ex{16};
  Block B1(32, 1), B2(32, 2);
  uint64_t t1, t2;
  fake_fail_alloc_in(1);   // the next allocation (the first block's workspace)
  CHECK(rfi_submit(s, a, &B1.blk, 0, &t1) == RFI_OK);
  rfi_result r{};
  CHECK(rfi_wait(s, t1, -1, &r) == RFI_OK);
  CHECK(r.status == RFI_E_NOMEM);
  CHECK(rfi_result_release(s, t1) == RFI_OK);
  // nothing of it ran: the stream continues as if it had not been submitted
  CHECK(rfi_submit(s, a, &B2.blk, 0, &t2) == RFI_OK);
  CHECK(rfi_wait(s, t2, -1, &r) == RFI_OK);
  CHECK(check_result(s, r, B2, ex.next(32), 16));
  rfi_session_destroy(s);
  std::printf("ok allocation_failure\n");
}

void partial_launch_failure() {
  fake_set_work_us(20000);
  rfi_session* s = make_session(2, 0);
  CHECK(s);
  const int a = open_stream(s, 16), b = open_stream(s, 16);
  Block B1(35, 1), B2(32, 2), C1(32, 3);
  uint64_t t1, t2, tc;
  // B1 is 2 full sub-intervals + 3 carry samples: sums/eigen, new carry,
  // clip; the clip launch (third launcher call) fails after two were enqueued
  fake_fail_launch_in(3);
  CHECK(rfi_submit(s, a, &B1.blk, 0, &t1) == RFI_OK);
  rfi_result r{};
  CHECK(rfi_wait(s, t1, -1, &r) == RFI_OK);
  CHECK(r.status == RFI_E_DEVICE);
  // it kept its slot until its enqueued work (two 20 ms items) had run
  CHECK(r.t_done_us - r.t_admit_us >= 35000.0);
  // its stream is failed; other streams are not
  CHECK(rfi_submit(s, a, &B2.blk, 0, &t2) == RFI_OK);
  CHECK(rfi_wait(s, t2, -1, &r) == RFI_OK && r.status == RFI_E_DEVICE);
  CHECK(rfi_submit(s, b, &C1.blk, 0, &tc) == RFI_OK);
  CHECK(rfi_wait(s, tc, -1, &r) == RFI_OK && r.status == RFI_OK);
  Expect ex{16};
  CHECK(check_result(s, r, C1, ex.next(32), 16));
  for (uint64_t t : {t1, t2}) CHECK(rfi_result_release(s, t) == RFI_OK);
  rfi_session_destroy(s);
  std::printf("ok partial_launch_failure\n");
}

void beam_stage() {
  fake_set_work_us(100);
  rfi_session* s = make_session(2, 0);
  CHECK(s);
  rfi_stream_config c{NB, NC, 16, 32, 12, 50, 3.0, nullptr, 1, 0, 1.0};
  int32_t id = -1;
  CHECK(rfi_stream_open(s, &c, &id) == RFI_OK);
  rfi_stream_config bad = c;
  bad.kappa_v = -1.0;
  int32_t id2 = -1;
  CHECK(rfi_stream_open(s, &bad, &id2) == RFI_E_INVALID);
  Expect ex{16};
  Block B1(37, 5), B2(30, 6);
  for (Block* b : {&B1, &B2}) {
    uint64_t t;
    CHECK(rfi_submit(s, id, &b->blk, 0, &t) == RFI_OK);
    rfi_result r{};
    CHECK(rfi_wait(s, t, -1, &r) == RFI_OK && r.status == RFI_OK);
    CHECK(r.v1 != nullptr && r.beam_mask != nullptr);
    const Expect::One e = ex.next(b->blk.nsamp);
    const size_t n = (size_t)e.nsub * NC;
    std::vector<uint8_t> mask(n + 1), bm(NB * n + 1);
    std::vector<float> v1(NB * n + 1);
    CHECK(rfi_result_copy(s, t, nullptr, nullptr, mask.data()) == RFI_OK);
    CHECK(rfi_result_copy_beams(s, t, v1.data(), bm.data()) == RFI_OK);
    for (int bb = 0; bb < NB; ++bb)
      for (size_t i = 0; i < n; ++i) CHECK(bm[bb * n + i] == mask[i]);   // the fake stage
    CHECK(rfi_result_release(s, t) == RFI_OK);
  }
  rfi_session_destroy(s);
  CHECK(fake_errors() == 0);
  std::printf("ok beam_stage\n");
}

void many_threads() {
  fake_set_work_us(50);
  rfi_session* s = make_session(3, 0);
  CHECK(s);
  std::atomic<int> bad{0};
  std::vector<std::thread> th;
  for (int w = 0; w < 4; ++w)
    th.emplace_back([&, w] {
      const int L = 8 + 3 * w;
      const int id = open_stream(s, L);
      if (id < 0) {
        bad++;
        return;
      }
      Expect ex{L};
      std::mt19937 g(77 + w);
      std::vector<std::unique_ptr<Block>> blocks;
      std::vector<uint64_t> tickets;
      std::vector<Expect::One> exp;
      for (int i = 0; i < 25; ++i) {
        const int64_t n = g() % 60;
        blocks.emplace_back(new Block(n, 1000 * w + i));
        uint64_t t;
        if (rfi_submit(s, id, &blocks.back()->blk, i, &t) != RFI_OK) {
          bad++;
          return;
        }
        tickets.push_back(t);
        exp.push_back(ex.next(n));
        if (i % 3 == 0) {   // wait on some right away, poll others later
          rfi_result r{};
          if (rfi_wait(s, t, -1, &r) != RFI_OK) bad++;
        }
      }
      for (size_t k = 0; k < tickets.size(); ++k) {
        rfi_result r{};
        while (rfi_poll(s, tickets[k], &r) == RFI_E_NOT_READY) std::this_thread::yield();
        if (!check_result(s, r, *blocks[k], exp[k], L)) bad++;
      }
      if (rfi_stream_close(s, id) != RFI_OK) bad++;
    });
  for (auto& t : th) t.join();
  CHECK(bad == 0);
  rfi_session_destroy(s);
  CHECK(fake_errors() == 0);
  std::printf("ok many_threads\n");
}

}  // namespace

int main() {
  order_and_carries();
  long_carries();
  budget_and_no_head_of_line();
  cancel_and_close();
  export_import();
  allocation_failure();
  partial_launch_failure();
  beam_stage();
  many_threads();
  std::printf(g_fail ? "SOME CHECKS FAILED\n" : "ALL OK\n");
  return g_fail ? 1 : 0;
}

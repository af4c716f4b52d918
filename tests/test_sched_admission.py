"""The serving loop's admission decision (`csrc/admit.h`, the function the
worker pool calls under its lock) driven by a fake executor on the CPU: a
discrete-event simulation of workers that hold grow-only buffers between
problems, with seeded arrivals, footprints up to the whole budget and
running times.  Checked: the reserved bytes never exceed the budget, every
request is admitted and finishes (no deadlock with all workers idle), and
the oldest request is passed over at most kMaxSkips times."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_00358_amd", "csrc")

DRIVER = r"""
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "admit.h"

using namespace hotrg;

struct Req {
  size_t foot, held;
  double arrive, dur;
  int skips;
};
struct Worker {
  size_t hold = 0;
  Req* run = nullptr;
  double end = 0;
};

int main(int argc, char** argv) {
  const unsigned seed = (unsigned)atoi(argv[1]);
  const int W = atoi(argv[2]);
  const int N = atoi(argv[3]);
  const size_t budget = 1000;
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<Req> reqs(N);
  double t = 0;
  for (int i = 0; i < N; ++i) {
    t += 0.3 * u(g);
    const double x = u(g);
    // mostly small problems, some up to the whole budget
    const size_t foot = 1 + (size_t)((budget - 1) * x * x * x);
    reqs[i] = {foot, (size_t)(foot * u(g)), t, 0.2 + 3.0 * u(g), 0};
  }
  std::deque<Req*> q;
  std::vector<Worker> w(W);
  size_t reserved = 0, peak = 0;
  int next = 0, done = 0, max_skips = 0;
  long rounds = 0;
  auto foot = [](Req* r) { return r->foot; };
  auto skips = [](Req* r) { return r->skips; };
  while (done < N) {
    double now = 1e300;
    if (next < N) now = reqs[next].arrive;
    for (auto& x : w)
      if (x.run) now = std::min(now, x.end);
    if (now == 1e300) {
      printf("deadlock: %zu queued, all workers idle\n", q.size());
      return 1;
    }
    for (auto& x : w)
      if (x.run && x.end <= now) {
        reserved -= x.run->foot + x.hold;  // its footprint and the buffers held before
        x.hold = x.run->held;              // what the context keeps afterwards
        reserved += x.hold;
        x.run = nullptr;
        ++done;
      }
    while (next < N && reqs[next].arrive <= now) q.push_back(&reqs[next++]);
    for (bool changed = true; changed;) {
      changed = false;
      for (auto& x : w) {
        if (x.run) continue;
        for (;;) {
          const AdmitChoice ch = admit_choice(q, foot, skips, reserved - x.hold, x.hold, budget);
          if (ch.action == ADMIT_RELEASE) {
            if (x.hold == 0) {
              printf("release with nothing held\n");
              return 1;
            }
            reserved -= x.hold;
            x.hold = 0;
            changed = true;
            continue;
          }
          if (ch.action == ADMIT_RUN) {
            if (ch.index > 0) ++q.front()->skips;
            Req* r = q[ch.index];
            q.erase(q.begin() + (long)ch.index);
            reserved += r->foot;
            if (reserved > budget) {
              printf("over budget: %zu > %zu\n", reserved, budget);
              return 1;
            }
            peak = std::max(peak, reserved);
            max_skips = std::max(max_skips, r->skips);
            x.run = r;
            x.end = now + r->dur;
            changed = true;
          }
          break;
        }
      }
    }
    if (++rounds > 100000000L) {
      printf("no progress\n");
      return 1;
    }
  }
  if (max_skips > kMaxSkips) {
    printf("oldest request passed over %d times\n", max_skips);
    return 1;
  }
  printf("ok done %d peak %zu max_skips %d\n", done, peak, max_skips);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("admit")
    src = d / "admit_sim.cpp"
    src.write_text(DRIVER)
    exe = d / "admit_sim"
    subprocess.run([gxx, "-std=c++17", "-O2", "-Wall", "-Werror", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True, capture_output=True, text=True)
    return str(exe)


@pytest.mark.parametrize("workers", [1, 4, 16])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_admission_invariants(driver, workers, seed):
    r = subprocess.run([driver, str(seed), str(workers), "600"], capture_output=True, text=True,
                       timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok done 600")

// Host symbolic stage of the thresholded block product C = A B (paper,
// section 3.2, equations 2 and 3): candidate columns, the block-norm bound,
// the kept pattern and the per-block product lists the device consumes.
#include <algorithm>
#include <atomic>
#include <thread>

#include "common.hpp"

namespace vbcsr {

namespace {

// Scratch of one worker: dense per-atom accumulators, reset after each row.
struct RowScratch {
  std::vector<double> acc;
  std::vector<int32_t> slot;   // -1, or position of column j in `cols`
  std::vector<int32_t> cols;
  std::vector<int64_t> nprod;
  explicit RowScratch(int32_t n) : acc(n, 0.0), slot(n, -1) {}
};

// Candidates of row i with their bound and product count; `cols` sorted.
void scan_row(int32_t i, const int64_t *arp, const int32_t *aci, const double *an,
              const int64_t *brp, const int32_t *bci, const double *bn, RowScratch &w) {
  w.cols.clear();
  for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
    const int32_t k = aci[ka];
    for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) {
      const int32_t j = bci[kb];
      if (w.slot[j] < 0) {
        w.slot[j] = (int32_t)w.cols.size();
        w.cols.push_back(j);
      }
      if (an) w.acc[j] += an[ka] * bn[kb];
    }
  }
  std::sort(w.cols.begin(), w.cols.end());
}

void clear_row(RowScratch &w) {
  for (int32_t j : w.cols) {
    w.slot[j] = -1;
    w.acc[j] = 0.0;
  }
}

unsigned worker_count(int32_t n) {
  return n < 4096 ? 1u : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
}

// body(worker, r0, r1) over chunks of rows, nt workers (worker 0 is the caller).
template <typename F>
void parallel_rows(int32_t n, unsigned nt, F &&body) {
  const int32_t chunk = 256;
  std::atomic<int32_t> next{0};
  auto work = [&](unsigned t) {
    for (;;) {
      const int32_t r0 = next.fetch_add(chunk);
      if (r0 >= n) break;
      body(t, r0, std::min(n, r0 + chunk));
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(work, t);
  work(0);
  for (auto &x : th) x.join();
}

}  // namespace

void spgemm_symbolic(int32_t n, const int32_t *b, const int64_t *arp, const int32_t *aci,
                     const int64_t *apos, const double *an, const int64_t *brp,
                     const int32_t *bci, const int64_t *bpos, const double *bn, double eps,
                     SpgemmPlan &out) {
  const bool thr = an && bn;
  std::vector<int64_t> kept(n, 0), prods(n, 0), cands(n, 0);
  std::vector<double> fl(n, 0.0);
  const unsigned nw = worker_count(n);
  std::vector<RowScratch> ws;
  ws.reserve(nw);
  for (unsigned t = 0; t < nw; ++t) ws.emplace_back(n);

  // pass 1: counts per row
  parallel_rows(n, nw, [&](unsigned t, int32_t r0, int32_t r1) {
    RowScratch &w = ws[t];
    for (int32_t i = r0; i < r1; ++i) {
      scan_row(i, arp, aci, thr ? an : nullptr, brp, bci, bn, w);
      cands[i] = (int64_t)w.cols.size();
      // products per candidate, counted by column
      w.nprod.assign(w.cols.size(), 0);
      for (size_t c = 0; c < w.cols.size(); ++c) w.slot[w.cols[c]] = (int32_t)c;
      for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
        const int32_t k = aci[ka];
        for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) w.nprod[w.slot[bci[kb]]]++;
      }
      int64_t nk = 0, np = 0;
      double f = 0.0;
      for (size_t c = 0; c < w.cols.size(); ++c) {
        const int32_t j = w.cols[c];
        if (thr && w.acc[j] < eps) continue;
        ++nk;
        np += w.nprod[c];
      }
      // flops: every product of a kept block, 2 b_i b_k b_j
      for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
        const int32_t k = aci[ka];
        for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) {
          const int32_t j = bci[kb];
          if (thr && w.acc[j] < eps) continue;
          f += 2.0 * b[i] * b[k] * b[j];
        }
      }
      kept[i] = nk;
      prods[i] = np;
      fl[i] = f;
      clear_row(w);
    }
  });

  out.row_ptr.assign((size_t)n + 1, 0);
  std::vector<int64_t> prow((size_t)n + 1, 0), vrow((size_t)n + 1, 0);
  out.candidates = 0;
  out.flops = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    out.row_ptr[i + 1] = out.row_ptr[i] + kept[i];
    prow[i + 1] = prow[i] + prods[i];
    out.candidates += cands[i];
    out.flops += fl[i];
  }
  const int64_t nC = out.row_ptr[n], nP = prow[n];
  // every entry below is written exactly once by pass 2 (and the final
  // offsets), so the buffers are not cleared first
  out.oi.resize(nC);
  out.oj.resize(nC);
  out.bound.resize(nC);
  out.obase.resize(nC + 1);
  out.pptr.resize(nC + 1);
  out.pa.resize(nP);
  out.pb.resize(nP);
  // value offsets need the running sum over rows of b_i * sum b_j
  std::vector<int64_t> vsum(n, 0);

  // pass 2: fill columns, bounds, product ranges and product lists
  parallel_rows(n, nw, [&](unsigned t, int32_t r0, int32_t r1) {
    RowScratch &w = ws[t];
    for (int32_t i = r0; i < r1; ++i) {
      scan_row(i, arp, aci, thr ? an : nullptr, brp, bci, bn, w);
      int64_t c = out.row_ptr[i];
      // slot[j] <- index of kept block (global), or -2 for dropped candidates
      for (int32_t j : w.cols) {
        if (thr && w.acc[j] < eps) {
          w.slot[j] = -2;
          continue;
        }
        w.slot[j] = (int32_t)(c - out.row_ptr[i]);
        out.oi[c] = i;
        out.oj[c] = j;
        out.bound[c] = thr ? w.acc[j] : 0.0;
        ++c;
      }
      // product counts of the kept blocks -> ranges (relative to the row)
      const int64_t nk = out.row_ptr[i + 1] - out.row_ptr[i];
      w.nprod.assign(nk + 1, 0);
      for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
        const int32_t k = aci[ka];
        for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) {
          const int32_t s = w.slot[bci[kb]];
          if (s >= 0) w.nprod[s + 1]++;
        }
      }
      for (int64_t q = 0; q < nk; ++q) w.nprod[q + 1] += w.nprod[q];
      int64_t vs = 0;
      for (int64_t q = 0; q < nk; ++q) {
        const int64_t cc = out.row_ptr[i] + q;
        out.pptr[cc] = prow[i] + w.nprod[q];
        out.obase[cc] = vs;  // relative to the row for now
        vs += (int64_t)b[i] * b[out.oj[cc]];
      }
      vsum[i] = vs;
      // products in A's stored order of k
      for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
        const int32_t k = aci[ka];
        for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) {
          const int32_t s = w.slot[bci[kb]];
          if (s < 0) continue;
          const int64_t pos = prow[i] + w.nprod[s]++;
          out.pa[pos] = apos[ka] << 8 | (int64_t)b[k];
          out.pb[pos] = bpos[kb];
        }
      }
      clear_row(w);
    }
  });
  int64_t base = 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t c = out.row_ptr[i]; c < out.row_ptr[i + 1]; ++c) out.obase[c] += base;
    base += vsum[i];
  }
  out.obase[nC] = base;
  out.pptr[nC] = nP;
}

}  // namespace vbcsr

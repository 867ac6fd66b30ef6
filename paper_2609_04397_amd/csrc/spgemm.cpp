// Host symbolic stage of the thresholded block product C = A B (paper,
// section 3.2, equations 2 and 3): candidate columns, the block-norm bound,
// the kept pattern and the per-block product lists the device consumes.
#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>

#include "common.hpp"

namespace vbcsr {

namespace {

// Scratch of one worker: dense per-atom accumulators, reset after each row.
struct RowScratch {
  std::vector<double> acc;     // bound U_ij of candidate j
  std::vector<int32_t> slot;   // -1, or position of column j in `cols`
  std::vector<int32_t> nprod;  // products of candidate j
  std::vector<int64_t> bksum;  // sum of b_k over the products of candidate j
  std::vector<int32_t> cols;
  std::vector<uint64_t> bits;  // candidate bitmap over [jmin, jmax]
  explicit RowScratch(int32_t n) : acc(n, 0.0), slot(n, -1), nprod(n, 0), bksum(n, 0) {}
};

// Put the row's candidates in ascending order: a bitmap scan when the span
// of their columns is small next to their count (linear in both), else a
// comparison sort.
void order_candidates(RowScratch &w, int32_t jmin, int32_t jmax) {
  const size_t nc = w.cols.size();
  if (nc < 2) return;
  const int64_t span = (int64_t)jmax - jmin + 1;
  if (span > 256 * (int64_t)nc) {
    std::sort(w.cols.begin(), w.cols.end());
    return;
  }
  const size_t nw = (size_t)((span + 63) >> 6);
  w.bits.assign(nw, 0);
  for (int32_t j : w.cols) w.bits[(size_t)(j - jmin) >> 6] |= uint64_t(1) << ((j - jmin) & 63);
  w.cols.clear();
  for (size_t q = 0; q < nw; ++q)
    for (uint64_t v = w.bits[q]; v; v &= v - 1)
      w.cols.push_back(jmin + (int32_t)(q << 6) + __builtin_ctzll(v));
}

// The kept blocks of one row, ascending in j, from the counting pass.
struct RowKept {
  std::vector<int32_t> col;
  std::vector<double> bound;
  std::vector<int32_t> nprod;
};

unsigned worker_count(int32_t n) {
  return n < 4096 ? 1u : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
}

// body(worker, r0, r1) over chunks of rows, nt workers (worker 0 is the
// caller).  A worker thread that cannot be started leaves its share to the
// others; an exception thrown by body stops the remaining chunks and is
// rethrown here once every thread has joined.
template <typename F>
void parallel_rows_w(int32_t n, unsigned nt, F &&body) {
  const int64_t chunk = 256;
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&](unsigned t) {
    try {
      for (;;) {
        const int64_t r0 = next.fetch_add(chunk);
        if (r0 >= n) break;
        body(t, (int32_t)r0, (int32_t)std::min<int64_t>(n, r0 + chunk));
      }
    } catch (...) {
      std::lock_guard<std::mutex> lock(mu);
      if (!err) err = std::current_exception();
      next.store(n);
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) {
    try {
      th.emplace_back(work, t);
    } catch (...) {
      break;
    }
  }
  work(0);
  for (auto &x : th) x.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace

void spgemm_symbolic(int32_t n, const int32_t *b, const int64_t *arp, const int32_t *aci,
                     const int64_t *apos, const double *an, const int64_t *brp,
                     const int32_t *bci, const int64_t *bpos, const double *bn, double eps,
                     SpgemmPlan &out) {
  const bool thr = an && bn;
  std::vector<int64_t> prods(n, 0), cands(n, 0);
  std::vector<double> fl(n, 0.0);
  std::vector<RowKept> rk((size_t)n);
  const unsigned nw = worker_count(n);
  std::vector<RowScratch> ws;
  ws.reserve(nw);
  for (unsigned t = 0; t < nw; ++t) ws.emplace_back(n);

  // pass 1, one sweep over the products of each row: candidates, their
  // bounds (summed over k in A's stored order, then B's), product counts
  // and sum of b_k; the kept ones are stored ascending in j
  parallel_rows_w(n, nw, [&](unsigned t, int32_t r0, int32_t r1) {
    RowScratch &w = ws[t];
    for (int32_t i = r0; i < r1; ++i) {
      w.cols.clear();
      int32_t jmin = n, jmax = -1;
      for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
        const int32_t k = aci[ka];
        for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) {
          const int32_t j = bci[kb];
          if (w.slot[j] < 0) {
            w.slot[j] = (int32_t)w.cols.size();
            w.cols.push_back(j);
            jmin = std::min(jmin, j);
            jmax = std::max(jmax, j);
          }
          if (thr) w.acc[j] += an[ka] * bn[kb];
          ++w.nprod[j];
          w.bksum[j] += b[k];
        }
      }
      order_candidates(w, jmin, jmax);
      cands[i] = (int64_t)w.cols.size();
      RowKept &r = rk[i];
      int64_t np = 0;
      double f = 0.0;
      for (int32_t j : w.cols) {
        if (!(thr && w.acc[j] < eps)) {
          r.col.push_back(j);
          r.bound.push_back(thr ? w.acc[j] : 0.0);
          r.nprod.push_back(w.nprod[j]);
          np += w.nprod[j];
          // flops: every product of a kept block, 2 b_i b_k b_j
          f += 2.0 * b[i] * (double)w.bksum[j] * b[j];
        }
        w.slot[j] = -1;
        w.acc[j] = 0.0;
        w.nprod[j] = 0;
        w.bksum[j] = 0;
      }
      prods[i] = np;
      fl[i] = f;
    }
  });

  out.row_ptr.assign((size_t)n + 1, 0);
  std::vector<int64_t> prow((size_t)n + 1, 0);
  out.candidates = 0;
  out.flops = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    out.row_ptr[i + 1] = out.row_ptr[i] + (int64_t)rk[i].col.size();
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

  // pass 2: kept blocks, product ranges, and one more sweep to list the
  // products of the kept blocks in A's stored order of k
  parallel_rows_w(n, nw, [&](unsigned t, int32_t r0, int32_t r1) {
    RowScratch &w = ws[t];
    std::vector<int64_t> next;
    for (int32_t i = r0; i < r1; ++i) {
      RowKept &r = rk[i];
      const int64_t c0 = out.row_ptr[i], nk = (int64_t)r.col.size();
      next.resize(nk);
      int64_t vs = 0, p = prow[i];
      for (int64_t q = 0; q < nk; ++q) {
        const int32_t j = r.col[q];
        w.slot[j] = (int32_t)q;
        out.oi[c0 + q] = i;
        out.oj[c0 + q] = j;
        out.bound[c0 + q] = r.bound[q];
        out.pptr[c0 + q] = p;
        out.obase[c0 + q] = vs;  // relative to the row for now
        next[q] = p;
        p += r.nprod[q];
        vs += (int64_t)b[i] * b[j];
      }
      vsum[i] = vs;
      for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
        const int32_t k = aci[ka];
        for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) {
          const int32_t s = w.slot[bci[kb]];
          if (s < 0) continue;
          const int64_t pos = next[s]++;
          out.pa[pos] = apos[ka] << 8 | (int64_t)b[k];
          out.pb[pos] = bpos[kb];
        }
      }
      for (int32_t j : r.col) w.slot[j] = -1;
      std::vector<int32_t>().swap(r.col);
      std::vector<double>().swap(r.bound);
      std::vector<int32_t>().swap(r.nprod);
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

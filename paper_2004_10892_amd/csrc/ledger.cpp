// Slice ledger: which slice ranges of one contraction are done, and their
// FP64 partial sums.  The slices are independent subtasks (Sec. 2.4) whose
// sum is the result (Eq. 4); a lost range is contracted again alone.  Host
// code over the public calls only (qbe_plan_stats, qbe_contract_slices).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/qbe.h"

namespace qbe {
void set_error(const std::string& s);
}
using qbe::set_error;

struct qbe_ledger {
  int64_t n_slices = 0, range_size = 0;
  uint64_t tag = 0;
  std::vector<uint8_t> done;        // per range
  std::vector<double> partial;      // per range: re, im
  int64_t n_ranges() const { return (int64_t)done.size(); }
};

namespace {

const char kMagic[8] = {'Q', 'B', 'E', 'L', 'D', 'G', '0', '1'};

#define LEDGER_REQUIRE(cond, msg) \
  do {                            \
    if (!(cond)) {                \
      set_error(msg);             \
      return QBE_ERR_INVALID_ARG; \
    }                             \
  } while (0)

// Every entry point: no exception crosses the ABI.
template <class F>
int guarded(F f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return QBE_ERR_OOM;
  } catch (const std::exception& e) {
    set_error(std::string("internal: ") + e.what());
    return QBE_ERR_INTERNAL;
  } catch (...) {
    set_error("internal: unknown exception");
    return QBE_ERR_INTERNAL;
  }
}

int64_t ranges_of(int64_t n_slices, int64_t range_size) { return (n_slices - 1) / range_size + 1; }

void bounds(const qbe_ledger& l, int64_t i, int64_t* b, int64_t* e) {
  *b = i * l.range_size;
  *e = *b + std::min(l.range_size, l.n_slices - *b);
}

}  // namespace

int qbe_ledger_create(int64_t n_slices, int64_t range_size, uint64_t tag, qbe_ledger** out) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(out, "NULL argument");
    *out = nullptr;
    LEDGER_REQUIRE(n_slices >= 1 && range_size >= 1, "ledger needs n_slices >= 1 and range_size >= 1");
    auto l = std::make_unique<qbe_ledger>();
    l->n_slices = n_slices;
    l->range_size = range_size;
    l->tag = tag;
    const int64_t n = ranges_of(n_slices, range_size);
    l->done.assign(n, 0);
    l->partial.assign(2 * n, 0.0);
    *out = l.release();
    return (int)QBE_OK;
  });
}

int qbe_ledger_destroy(qbe_ledger* ledger) {
  delete ledger;
  return QBE_OK;
}

int qbe_ledger_info(const qbe_ledger* l, int64_t* n_slices, int64_t* range_size, uint64_t* tag, int64_t* n_ranges,
                    int64_t* n_done) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(l, "NULL ledger");
    if (n_slices) *n_slices = l->n_slices;
    if (range_size) *range_size = l->range_size;
    if (tag) *tag = l->tag;
    if (n_ranges) *n_ranges = l->n_ranges();
    if (n_done) {
      int64_t k = 0;
      for (uint8_t d : l->done) k += d;
      *n_done = k;
    }
    return (int)QBE_OK;
  });
}

int qbe_ledger_next(const qbe_ledger* l, int64_t* idx_out, int64_t* s_begin_out, int64_t* s_end_out) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(l && idx_out && s_begin_out && s_end_out, "NULL argument");
    *idx_out = -1;
    *s_begin_out = *s_end_out = 0;
    for (int64_t i = 0; i < l->n_ranges(); ++i)
      if (!l->done[i]) {
        *idx_out = i;
        bounds(*l, i, s_begin_out, s_end_out);
        break;
      }
    return (int)QBE_OK;
  });
}

int qbe_ledger_record(qbe_ledger* l, int64_t idx, const double* partial) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(l && partial, "NULL argument");
    LEDGER_REQUIRE(0 <= idx && idx < l->n_ranges(), "range index out of range");
    LEDGER_REQUIRE(!l->done[idx], "range " + std::to_string(idx) + " is already recorded");
    LEDGER_REQUIRE(std::isfinite(partial[0]) && std::isfinite(partial[1]),
                   "partial sum of range " + std::to_string(idx) + " is not finite");
    l->partial[2 * idx] = partial[0];
    l->partial[2 * idx + 1] = partial[1];
    l->done[idx] = 1;
    return (int)QBE_OK;
  });
}

int qbe_ledger_drop(qbe_ledger* l, int64_t idx) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(l, "NULL ledger");
    LEDGER_REQUIRE(0 <= idx && idx < l->n_ranges(), "range index out of range");
    l->done[idx] = 0;
    l->partial[2 * idx] = l->partial[2 * idx + 1] = 0.0;
    return (int)QBE_OK;
  });
}

int qbe_ledger_get(const qbe_ledger* l, int64_t idx, int32_t* done_out, double* partial_out) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(l && done_out && partial_out, "NULL argument");
    LEDGER_REQUIRE(0 <= idx && idx < l->n_ranges(), "range index out of range");
    *done_out = l->done[idx];
    partial_out[0] = l->partial[2 * idx];
    partial_out[1] = l->partial[2 * idx + 1];
    return (int)QBE_OK;
  });
}

int qbe_ledger_run(qbe_ctx* ctx, const qbe_plan* plan, qbe_ledger* l, void* d_workspace, size_t ws_bytes,
                   int64_t max_ranges, int64_t* n_run_out) {
  return guarded([&]() -> int {
    if (n_run_out) *n_run_out = 0;
    LEDGER_REQUIRE(ctx && plan && l, "NULL argument");
    qbe_stats st;
    int rc = qbe_plan_stats(plan, &st);
    if (rc) return rc;
    LEDGER_REQUIRE(st.m >= 0 && st.m < 63 && (int64_t(1) << st.m) == l->n_slices,
                   "the plan's slice count 2^m differs from the ledger's n_slices");
    int64_t run = 0;
    for (int64_t i = 0; i < l->n_ranges() && (max_ranges < 0 || run < max_ranges); ++i) {
      if (l->done[i]) continue;
      int64_t b, e;
      bounds(*l, i, &b, &e);
      double part[2];
      rc = qbe_contract_slices(ctx, plan, b, e, d_workspace, ws_bytes, part, nullptr);
      if (rc) return rc;
      rc = qbe_ledger_record(l, i, part);
      if (rc) return rc;
      ++run;
      if (n_run_out) *n_run_out = run;
    }
    return (int)QBE_OK;
  });
}

int qbe_ledger_sum(const qbe_ledger* l, double* amp_out) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(l && amp_out, "NULL argument");
    int64_t pending = 0;
    for (uint8_t d : l->done) pending += !d;
    LEDGER_REQUIRE(pending == 0, std::to_string(pending) + " ranges pending");
    double re = 0.0, im = 0.0;
    for (int64_t i = 0; i < l->n_ranges(); ++i) {
      re += l->partial[2 * i];
      im += l->partial[2 * i + 1];
    }
    amp_out[0] = re;
    amp_out[1] = im;
    return (int)QBE_OK;
  });
}

int qbe_ledger_save(const qbe_ledger* l, const char* path) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(l && path, "NULL argument");
    std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "wb"), std::fclose);
    LEDGER_REQUIRE(f, std::string("cannot open ") + path + " for writing");
    const int64_t hdr[2] = {l->n_slices, l->range_size};
    bool ok = std::fwrite(kMagic, 1, 8, f.get()) == 8 && std::fwrite(hdr, 8, 2, f.get()) == 2 &&
              std::fwrite(&l->tag, 8, 1, f.get()) == 1;
    for (int64_t i = 0; ok && i < l->n_ranges(); ++i) {
      const int64_t d = l->done[i];
      ok = std::fwrite(&d, 8, 1, f.get()) == 1 && std::fwrite(&l->partial[2 * i], 8, 2, f.get()) == 2;
    }
    ok = std::fclose(f.release()) == 0 && ok;
    LEDGER_REQUIRE(ok, std::string("write to ") + path + " failed");
    return (int)QBE_OK;
  });
}

int qbe_ledger_load(const char* path, qbe_ledger** out) {
  return guarded([&]() -> int {
    LEDGER_REQUIRE(path && out, "NULL argument");
    *out = nullptr;
    std::unique_ptr<FILE, int (*)(FILE*)> f(std::fopen(path, "rb"), std::fclose);
    LEDGER_REQUIRE(f, std::string("cannot open ") + path);
    char magic[8];
    int64_t hdr[2];
    uint64_t tag;
    LEDGER_REQUIRE(std::fread(magic, 1, 8, f.get()) == 8 && std::memcmp(magic, kMagic, 8) == 0,
                   std::string(path) + " is not a slice ledger");
    LEDGER_REQUIRE(std::fread(hdr, 8, 2, f.get()) == 2 && std::fread(&tag, 8, 1, f.get()) == 1,
                   std::string(path) + " is truncated");
    LEDGER_REQUIRE(hdr[0] >= 1 && hdr[1] >= 1, std::string(path) + ": bad n_slices or range_size");
    const int64_t n = ranges_of(hdr[0], hdr[1]);
    // each range takes 24 bytes: the file must hold them, and nothing more
    const long at = std::ftell(f.get());
    LEDGER_REQUIRE(at >= 0 && std::fseek(f.get(), 0, SEEK_END) == 0, std::string(path) + ": cannot seek");
    const long size = std::ftell(f.get());
    LEDGER_REQUIRE(size >= at && (size - at) % 24 == 0 && (size - at) / 24 == n,
                   std::string(path) + ": size differs from its range count");
    LEDGER_REQUIRE(std::fseek(f.get(), at, SEEK_SET) == 0, std::string(path) + ": cannot seek");
    auto l = std::make_unique<qbe_ledger>();
    l->n_slices = hdr[0];
    l->range_size = hdr[1];
    l->tag = tag;
    l->done.assign(n, 0);
    l->partial.assign(2 * n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      int64_t d;
      double v[2];
      LEDGER_REQUIRE(std::fread(&d, 8, 1, f.get()) == 1 && std::fread(v, 8, 2, f.get()) == 2,
                     std::string(path) + " is truncated");
      LEDGER_REQUIRE(d == 0 || d == 1, std::string(path) + ": bad done flag at range " + std::to_string(i));
      LEDGER_REQUIRE(std::isfinite(v[0]) && std::isfinite(v[1]),
                     std::string(path) + ": non-finite value at range " + std::to_string(i));
      l->done[i] = (uint8_t)d;
      l->partial[2 * i] = v[0];
      l->partial[2 * i + 1] = v[1];
    }
    *out = l.release();
    return (int)QBE_OK;
  });
}

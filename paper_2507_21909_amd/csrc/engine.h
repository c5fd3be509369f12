// Host engine of the RG step: device arena, tensor contraction over labelled
// legs, and the state of one solve.
#pragma once
#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/trg.h"
#include "common.h"

namespace trg {

// Bump allocator over device chunks; mark/release gives stack-like scopes.
class Arena {
  public:
    explicit Arena(size_t cap = 0) : cap_(cap) {}
    ~Arena();
    void *alloc(size_t bytes);
    double *dalloc(size_t n) { return static_cast<double *>(alloc(n * sizeof(double))); }
    struct Mark { size_t chunk, used; };
    Mark mark() const;
    void release(const Mark &m);
    void reset() { release(Mark{0, 0}); }
    // frees every chunk (no allocation may be live, nor any kernel using one)
    void trim();
    size_t held() const { return total_; }
    void set_cap(size_t c) { cap_ = c; }
    // frozen: an allocation that needs a new chunk throws instead (graph capture)
    void freeze(bool f) { frozen_ = f; }

  private:
    struct Chunk { char *base; size_t cap, used; };
    std::vector<Chunk> chunks_;
    size_t cur_ = 0, total_ = 0, cap_ = 0;
    bool frozen_ = false;
};

// Device tensor: row-major, leftmost leg slowest.
struct DT {
    double *p = nullptr;
    std::vector<int> d;
    long n() const {
        long x = 1;
        for (int v : d) x *= v;
        return x;
    }
};

struct TimedGemm {
    hipEvent_t a, b;
    double flops;
};

struct Ctx {
    hipStream_t st;
    Arena *ar;
    Prec prec;
    // HIP events around selected GEMM launches (the coarse-graining GEMMs)
    bool timing = false;
    std::vector<TimedGemm> timed;
    // graph capture: nothing is read back to the host; iterative solves stop on
    // device flags and report failures in *dstatus
    bool capture = false;
    int *dstatus = nullptr;
    // sweeps eager solves took, keyed by (call order, count, m, n); solve_idx counts calls
    std::map<std::array<int, 4>, int> *sweep_log = nullptr;
    int solve_idx = 0;
};

// gemm() bracketed by HIP events on the context's stream when c.timing is set
void timed_gemm(Ctx &c, const GemmArgs &g, Prec prec);
// gemm_planes() likewise; flops = the contraction's algorithmic 2 M N K
void timed_planes(Ctx &c, const PlaneGemm &g, double flops);

DT talloc(Ctx &c, std::vector<int> dims);
DT permuted(Ctx &c, const DT &a, const std::string &la, const std::string &lt);
// out[lo] = alpha * sum a[la] b[lb] ; labels are single characters.
DT contract(Ctx &c, const DT &a, const std::string &la, const DT &b, const std::string &lb,
            const std::string &lo, Prec prec = P_FP64, double alpha = 1.0);

}  // namespace trg

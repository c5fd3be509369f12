// Device arena and the labelled tensor contraction used by the RG step.
//
// contract() evaluates out[lo] = sum a[la] b[lb] as one strided batched GEMM:
// labels shared by a, b and out are the batch, labels shared by a and b only
// are contracted, the rest are the rows (from a) and columns (from b).  An
// operand is permuted first only when one of its label groups is not a
// contiguous block of its memory layout; likewise the result is permuted only
// when out's layout cannot be written by the GEMM directly.
#include <algorithm>
#include <map>

#include "engine.h"

namespace trg {

Arena::~Arena() {
    for (auto &c : chunks_) (void)hipFree(c.base);
}

void *Arena::alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    while (cur_ < chunks_.size()) {
        Chunk &c = chunks_[cur_];
        if (c.used + bytes <= c.cap) {
            void *p = c.base + c.used;
            c.used += bytes;
            return p;
        }
        ++cur_;
        if (cur_ < chunks_.size()) chunks_[cur_].used = 0;
    }
    TRG_REQUIRE(!frozen_, -2,
                "graph capture: the workspace would grow (run one eager step of this method at these shapes first)");
    size_t want = std::max(bytes, size_t(256) << 20);
    if (cap_ && total_ + want > cap_) {
        want = bytes;
        TRG_REQUIRE(total_ + want <= cap_, -3, "workspace cap exceeded");
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(-3, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    chunks_.push_back(Chunk{static_cast<char *>(p), want, bytes});
    cur_ = chunks_.size() - 1;
    total_ += want;
    return p;
}

void Arena::trim() {
    for (auto &c : chunks_) (void)hipFree(c.base);
    chunks_.clear();
    cur_ = 0;
    total_ = 0;
}

Arena::Mark Arena::mark() const {
    if (chunks_.empty()) return Mark{0, 0};
    return Mark{cur_, chunks_[cur_].used};
}

void Arena::release(const Mark &m) {
    if (chunks_.empty()) return;
    cur_ = std::min(m.chunk, chunks_.size() - 1);
    chunks_[cur_].used = (m.chunk < chunks_.size()) ? m.used : 0;
    for (size_t i = cur_ + 1; i < chunks_.size(); ++i) chunks_[i].used = 0;
}

DT talloc(Ctx &c, std::vector<int> dims) {
    DT t;
    t.d = std::move(dims);
    t.p = c.ar->dalloc((size_t)std::max(1L, t.n()));
    return t;
}

static std::vector<int> perm_of(const std::string &from, const std::string &to) {
    std::vector<int> p(to.size());
    for (size_t i = 0; i < to.size(); ++i) {
        size_t k = from.find(to[i]);
        TRG_REQUIRE(k != std::string::npos, -1, "permute: label missing");
        p[i] = (int)k;
    }
    return p;
}

DT permuted(Ctx &c, const DT &a, const std::string &la, const std::string &lt) {
    TRG_REQUIRE(la.size() == a.d.size() && lt.size() == la.size(), -1, "permuted: rank mismatch");
    std::vector<int> p = perm_of(la, lt);
    std::vector<int> dims(lt.size());
    for (size_t i = 0; i < lt.size(); ++i) dims[i] = a.d[p[i]];
    DT t = talloc(c, dims);
    permute(a.p, t.p, a.d, p, c.st);
    return t;
}

namespace {
struct View {
    std::map<char, long> stride, dim;
};

View view_of(const std::vector<int> &d, const std::string &l) {
    View v;
    long s = 1;
    for (int i = (int)l.size() - 1; i >= 0; --i) {
        v.stride[l[i]] = s;
        v.dim[l[i]] = d[i];
        s *= d[i];
    }
    return v;
}

// a label group is usable as one GEMM index if it is a contiguous block in memory
bool group(const View &v, const std::string &g, long &size, long &stride) {
    size = 1;
    stride = 0;
    if (g.empty()) return true;
    for (char ch : g) size *= v.dim.at(ch);
    for (size_t i = 0; i + 1 < g.size(); ++i)
        if (v.stride.at(g[i]) != v.stride.at(g[i + 1]) * v.dim.at(g[i + 1])) return false;
    stride = v.stride.at(g.back());
    return true;
}
}  // namespace

DT contract(Ctx &c, const DT &a, const std::string &la, const DT &b, const std::string &lb,
            const std::string &lo, Prec prec, double alpha) {
    TRG_REQUIRE(la.size() == a.d.size() && lb.size() == b.d.size(), -1, "contract: rank/labels mismatch");
    std::map<char, int> dim;
    for (size_t i = 0; i < la.size(); ++i) dim[la[i]] = a.d[i];
    for (size_t i = 0; i < lb.size(); ++i) {
        auto it = dim.find(lb[i]);
        TRG_REQUIRE(it == dim.end() || it->second == b.d[i], -1, "contract: dim mismatch on " + std::string(1, lb[i]));
        dim[lb[i]] = b.d[i];
    }
    auto in = [](const std::string &s, char ch) { return s.find(ch) != std::string::npos; };
    std::string bat, fa, fb, ctr_a, ctr_b;
    for (char ch : lo) {
        TRG_REQUIRE(in(la, ch) || in(lb, ch), -1, "contract: output label not in inputs");
        if (in(la, ch) && in(lb, ch)) bat += ch;
        else if (in(la, ch)) fa += ch;
        else fb += ch;
    }
    for (char ch : la)
        if (in(lb, ch) && !in(lo, ch)) ctr_a += ch;
    for (char ch : lb)
        if (in(la, ch) && !in(lo, ch)) ctr_b += ch;
    for (char ch : la) TRG_REQUIRE(in(lb, ch) || in(lo, ch), -1, "contract: free label of a missing in out");
    for (char ch : lb) TRG_REQUIRE(in(la, ch) || in(lo, ch), -1, "contract: free label of b missing in out");

    DT A = a, B = b;
    std::string lA = la, lB = lb;
    // choose the contracted order that needs fewest operand permutes
    std::string ctr = ctr_a;
    {
        long s, t;
        View va = view_of(a.d, la), vb = view_of(b.d, lb);
        auto okA = [&](const std::string &k) { return group(va, bat, s, t) && group(va, fa, s, t) && group(va, k, s, t); };
        auto okB = [&](const std::string &k) { return group(vb, bat, s, t) && group(vb, k, s, t) && group(vb, fb, s, t); };
        int sa = okA(ctr_a) + okB(ctr_a), sb = okA(ctr_b) + okB(ctr_b);
        if (sb > sa) ctr = ctr_b;
        if (!okA(ctr)) {
            A = permuted(c, a, la, bat + fa + ctr);
            lA = bat + fa + ctr;
        }
        if (!okB(ctr)) {
            B = permuted(c, b, lb, bat + ctr + fb);
            lB = bat + ctr + fb;
        }
    }
    std::vector<int> odims;
    for (char ch : lo) odims.push_back(dim[ch]);
    DT out = talloc(c, odims);
    View vA = view_of(A.d, lA), vB = view_of(B.d, lB), vO = view_of(out.d, lo);
    long nb, sAb, sBb, sCb, M, sAr, N, sBn, K, sAk, sBk, sCr, sCn, tmp;
    group(vA, bat, nb, sAb);
    group(vA, fa, M, sAr);
    group(vA, ctr, K, sAk);
    group(vB, bat, tmp, sBb);
    group(vB, ctr, tmp, sBk);
    group(vB, fb, N, sBn);
    bool direct = group(vO, bat, tmp, sCb) && group(vO, fa, tmp, sCr) && group(vO, fb, tmp, sCn);
    DT tgt = out;
    if (!direct) {
        std::vector<int> td;
        for (char ch : bat + fa + fb) td.push_back(dim[ch]);
        tgt = talloc(c, td);
        View vT = view_of(tgt.d, bat + fa + fb);
        group(vT, bat, tmp, sCb);
        group(vT, fa, tmp, sCr);
        group(vT, fb, tmp, sCn);
    }
    GemmArgs g{};
    g.M = (int)M; g.N = (int)N; g.K = (int)K; g.batch = (int)nb;
    g.A = A.p; g.sAr = sAr; g.sAk = sAk; g.sAb = sAb;
    g.B = B.p; g.sBk = sBk; g.sBn = sBn; g.sBb = sBb;
    g.C = tgt.p; g.sCr = sCr; g.sCn = sCn; g.sCb = sCb;
    g.alpha = alpha; g.beta = 0.0;
    const long tiles = ((M + 63) / 64) * ((N + 63) / 64) * nb;
    if (K == 0) {
        fill(tgt.p, (size_t)tgt.n(), 0.0, c.st);
    } else if (tiles < 512 && K >= 8192 && K % 2048 == 0) {
        // split K: few output tiles over a long contraction would leave most CUs
        // idle; the slices are added in a fixed order afterwards
        long splits = 1;
        while (splits < 1024 && tiles * splits < 1024 && K % (2 * splits * 1024) == 0 && nb * splits * 2 <= 65535)
            splits *= 2;
        double *w = c.ar->dalloc((size_t)nb * splits * M * N);
        GemmArgs h = g;
        h.K = (int)(K / splits);
        h.inner = (int)splits; h.sAi = h.K * sAk; h.sBi = h.K * sBk;
        h.C = w; h.sCr = N; h.sCn = 1; h.sCb = splits * M * N; h.sCi = M * N;
        gemm(h, prec, c.st);
        for (long b = 0; b < nb; ++b)
            sum_slices(w + b * splits * M * N, (int)splits, M, N, tgt.p + b * sCb, sCr, sCn, c.st);
    } else {
        gemm(g, prec, c.st);
    }
    if (!direct) permute(tgt.p, out.p, tgt.d, perm_of(bat + fa + fb, lo), c.st);
    return out;
}

void timed_gemm(Ctx &c, const GemmArgs &g, Prec prec) {
    if (!c.timing) {
        gemm(g, prec, c.st);
        return;
    }
    TimedGemm t;
    TRG_HIP_CHECK(hipEventCreate(&t.a));
    TRG_HIP_CHECK(hipEventCreate(&t.b));
    gemm(g, prec, c.st, t.a, t.b);   // the launch stamps both events (kernel start, end)
    t.flops = 2.0 * g.M * (double)g.N * g.K * g.batch * std::max(1, g.inner);
    c.timed.push_back(t);
}

void timed_planes(Ctx &c, const PlaneGemm &g, double flops) {
    if (!c.timing) {
        gemm_planes(g, c.st);
        return;
    }
    TimedGemm t;
    TRG_HIP_CHECK(hipEventCreate(&t.a));
    TRG_HIP_CHECK(hipEventCreate(&t.b));
    gemm_planes(g, c.st, t.a, t.b);
    t.flops = flops;
    c.timed.push_back(t);
}

void gemm(const GemmArgs &g, Prec prec, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (prec == P_FP64) gemm_f64(g, st, ev0, ev1);
    else gemm_mixed(g, (int)prec, st, ev0, ev1);
}

}  // namespace trg

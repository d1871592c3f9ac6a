// CPU model of the register-tiled pass engine (a host-logic test; no GPU).
//
// It runs the library's own host planner (compile_batch, compiled here from
// the library source) and replays every planned pass the way the kernels move
// data: 2^rb registers per thread in the pass's layouts, layout changes
// through a swizzled LDS array that is poisoned with NaN before each exchange,
// gates applied on register indices ka/kb.  States, expectation values and
// gradients are compared with a plain op-by-op state-vector reference written
// here (the gradient against central differences of it).  Structural checks:
// every layout is a permutation of the tile bits with consistent bit tables,
// targets sit on the register bits the op names, layout markers chain, and
// each pass ends in the layout it declares.
#include "sv_batch.hip"
#include <complex>
#include <cstdio>
#include <random>
#include <cassert>

using cd = std::complex<double>;

static uint32_t swz_h(uint32_t l) { return l ^ (((l >> 4) ^ (l >> 8) ^ (l >> 12)) & 15u); }

// ---------------- reference: dense per-op application --------------------
static void gate2(int g, double th, const double* mat, cd u[4])
{
    const double c = cos(th / 2), s = sin(th / 2), r = M_SQRT1_2;
    switch (g) {
    case SV_X: u[0] = 0; u[1] = 1; u[2] = 1; u[3] = 0; break;
    case SV_Y: u[0] = 0; u[1] = cd(0, -1); u[2] = cd(0, 1); u[3] = 0; break;
    case SV_Z: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = -1; break;
    case SV_H: u[0] = r; u[1] = r; u[2] = r; u[3] = -r; break;
    case SV_S: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = cd(0, 1); break;
    case SV_T: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = std::polar(1.0, M_PI / 4); break;
    case SV_RX: u[0] = c; u[1] = cd(0, -s); u[2] = cd(0, -s); u[3] = c; break;
    case SV_RY: u[0] = c; u[1] = -s; u[2] = s; u[3] = c; break;
    case SV_RZ: u[0] = cd(c, -s); u[1] = 0; u[2] = 0; u[3] = cd(c, s); break;
    case SV_PHASE: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = std::polar(1.0, th); break;
    case SV_U2: for (int k = 0; k < 4; ++k) u[k] = cd(mat[2 * k], mat[2 * k + 1]); break;
    default: assert(0);
    }
}

static void ref_apply(std::vector<cd>& psi, int n, const sv_op& o, const std::vector<double>& params)
{
    const double th = o.param_index >= 0 ? params[o.param_index] : o.value;
    const int nc = o.n_controls, nt = o.n_targets;
    uint64_t cm = 0;
    for (int j = 0; j < nc; ++j) cm |= 1ull << o.qubits[j];
    const uint64_t N = 1ull << n;
    if (nt == 1) {
        cd u[4];
        gate2(o.gate, th, o.matrix, u);
        const int t = o.qubits[nc];
        for (uint64_t x = 0; x < N; ++x) {
            if ((x >> t) & 1) continue;
            if ((x & cm) != cm) continue;
            const uint64_t y = x | (1ull << t);
            const cd a = psi[x], b = psi[y];
            psi[x] = u[0] * a + u[1] * b;
            psi[y] = u[2] * a + u[3] * b;
        }
    } else {
        const int ta = o.qubits[nc], tb = o.qubits[nc + 1];  // ta = matrix MSB
        cd U[16];
        if (o.gate == SV_SWAP) {
            for (int k = 0; k < 16; ++k) U[k] = 0;
            U[0] = U[6] = U[9] = U[15] = 1;
        } else
            for (int k = 0; k < 16; ++k) U[k] = cd(o.matrix[2 * k], o.matrix[2 * k + 1]);
        for (uint64_t x = 0; x < N; ++x) {
            if (((x >> ta) & 1) || ((x >> tb) & 1)) continue;
            if ((x & cm) != cm) continue;
            const uint64_t ix[4] = {x, x | (1ull << tb), x | (1ull << ta), x | (1ull << ta) | (1ull << tb)};
            cd v[4], w[4];
            for (int k = 0; k < 4; ++k) v[k] = psi[ix[k]];
            for (int r = 0; r < 4; ++r) {
                w[r] = 0;
                for (int c = 0; c < 4; ++c) w[r] += U[4 * r + c] * v[c];
            }
            for (int k = 0; k < 4; ++k) psi[ix[k]] = w[k];
        }
    }
}

static double obs_val(uint64_t x, int n, int kind)
{
    if (kind == 1) return n - 2 * __builtin_popcountll(x);
    const uint64_t m = n > 1 ? ((1ull << (n - 1)) - 1) : 0;
    return (n - 1) - 2 * __builtin_popcountll((x ^ (x >> 1)) & m);
}

static double ref_energy(int n, const std::vector<sv_op>& ops, const std::vector<double>& params, int kind,
                         std::vector<cd>* out = nullptr)
{
    std::vector<cd> psi(1ull << n, 0.0);
    psi[0] = 1;
    for (auto& o : ops) ref_apply(psi, n, o, params);
    double e = 0;
    for (uint64_t x = 0; x < psi.size(); ++x) e += obs_val(x, n, kind) * std::norm(psi[x]);
    if (out) *out = psi;
    return e;
}

// ---------------- emulation of the kernels -------------------------------
static int errors = 0;
static long pairc_lane = 0, pairc_reg = 0;  // two-branch ops replayed, by selector placement
static long gated_ops = 0;                  // one-target ops with controls outside the tile, per tile
static long tsel_ops = 0;                   // tile-selected fused ops replayed, per tile
static long run_members = 0;                // subset phases replayed as members of a per-target run
#define CHECK(c, ...) do { if (!(c)) { ++errors; if (errors < 20) { printf("FAIL %s:%d ", __FILE__, __LINE__); printf(__VA_ARGS__); printf("\n"); } } } while (0)

static void gate2x2_h(const FCoefSpec& f, const double* params, cd u[4])
{
    const double th = f.pidx >= 0 ? params[f.pidx] : f.value;
    const double ch = cos(th / 2), sh = sin(th / 2);
    switch (f.gate) {
    case SV_RX: u[0] = ch; u[1] = cd(0, -sh); u[2] = cd(0, -sh); u[3] = ch; break;
    case SV_RY: u[0] = ch; u[1] = -sh; u[2] = sh; u[3] = ch; break;
    case SV_RZ: u[0] = cd(ch, -sh); u[1] = 0; u[2] = 0; u[3] = cd(ch, sh); break;
    case SV_PHASE: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = std::polar(1.0, th); break;
    default: for (int k = 0; k < 4; ++k) u[k] = cd(f.fixed[2 * k], f.fixed[2 * k + 1]); break;
    }
}

static long rfuse_ops = 0;  // reverse pairs replayed, per tile

static void coef_eval(const FCoefSpec& s, const std::vector<FCoefSpec>& fac, const double* params, double* c)
{
    if (s.out_diag == 4) {
        // reverse pair A then B: B A, then B G B^dagger for A's generator G
        CHECK(s.nfactor == 2, "reverse pair with %d factors", s.nfactor);
        cd a[4], b[4];
        gate2x2_h(fac[s.factor_begin], params, a);
        gate2x2_h(fac[s.factor_begin + 1], params, b);
        auto mul = [](const cd* x, const cd* y, cd* r) {
            r[0] = x[0] * y[0] + x[1] * y[2];
            r[1] = x[0] * y[1] + x[1] * y[3];
            r[2] = x[2] * y[0] + x[3] * y[2];
            r[3] = x[2] * y[1] + x[3] * y[3];
        };
        cd ba[4];
        mul(b, a, ba);
        for (int q = 0; q < 4; ++q) { c[2 * q] = ba[q].real(); c[2 * q + 1] = ba[q].imag(); }
        for (int q = 8; q < 16; ++q) c[q] = 0;
        if (s.branch > 0) {
            cd g[4] = {0, 0, 0, 0};
            switch (s.branch - 1) {
            case GEN_X: g[1] = 1; g[2] = 1; break;
            case GEN_Y: g[1] = cd(0, -1); g[2] = cd(0, 1); break;
            case GEN_Z: g[0] = 1; g[3] = -1; break;
            default: g[3] = 1; break;
            }
            const cd bd[4] = {std::conj(b[0]), std::conj(b[2]), std::conj(b[1]), std::conj(b[3])};
            cd t[4], m[4];
            mul(g, bd, t);
            mul(b, t, m);
            for (int q = 0; q < 4; ++q) { c[8 + 2 * q] = m[q].real(); c[8 + 2 * q + 1] = m[q].imag(); }
        }
        return;
    }
    if (s.nfactor > 0 && s.out_diag == 3) {
        // one product per subset of the op's out-of-tile bits: the list of the
        // mask's set bits, entry e taking bit list[k] when bit k of e is set
        std::vector<int> bits;
        for (int q = 0; q < 32; ++q)
            if (((uint32_t)s.branch >> q) & 1u) bits.push_back(q);
        CHECK(!bits.empty() && (int)bits.size() <= kMaxTileSelBits, "tile-selected mask of %zu bits", bits.size());
        for (int e = 0; e < (1 << bits.size()); ++e) {
            uint32_t held = 0;
            for (size_t k = 0; k < bits.size(); ++k)
                if ((e >> k) & 1) held |= 1u << bits[k];
            cd m[4] = {1, 0, 0, 1};
            for (int k = 0; k < s.nfactor; ++k) {
                const FCoefSpec& fk = fac[s.factor_begin + k];
                CHECK(((uint32_t)fk.branch & ~(uint32_t)s.branch) == 0, "factor bits outside the op's mask");
                if (((uint32_t)fk.branch & held) != (uint32_t)fk.branch) continue;
                cd g[4], r[4];
                gate2x2_h(fk, params, g);
                r[0] = g[0] * m[0] + g[1] * m[2];
                r[1] = g[0] * m[1] + g[1] * m[3];
                r[2] = g[2] * m[0] + g[3] * m[2];
                r[3] = g[2] * m[1] + g[3] * m[3];
                for (int q = 0; q < 4; ++q) m[q] = r[q];
            }
            for (int q = 0; q < 4; ++q) { c[8 * e + 2 * q] = m[q].real(); c[8 * e + 2 * q + 1] = m[q].imag(); }
        }
        return;
    }
    if (s.nfactor > 0) {
        cd mm[2][4] = {{1, 0, 0, 1}, {1, 0, 0, 1}};
        for (int k = 0; k < s.nfactor; ++k) {
            const FCoefSpec& fk = fac[s.factor_begin + k];
            const int br = s.out_diag == 2 ? fk.branch : 1;
            CHECK(br >= 1 && br <= 3, "factor branch %d", br);
            cd g[4];
            gate2x2_h(fk, params, g);
            for (int w = 0; w < 2; ++w) {
                if (!((br >> w) & 1)) continue;
                cd* m = mm[w];
                cd r[4];
                r[0] = g[0] * m[0] + g[1] * m[2];
                r[1] = g[0] * m[1] + g[1] * m[3];
                r[2] = g[2] * m[0] + g[3] * m[2];
                r[3] = g[2] * m[1] + g[3] * m[3];
                for (int q = 0; q < 4; ++q) m[q] = r[q];
            }
        }
        const cd* m = mm[0];
        if (s.out_diag == 2) {
            for (int w = 0; w < 2; ++w)
                for (int q = 0; q < 4; ++q) { c[8 * w + 2 * q] = mm[w][q].real(); c[8 * w + 2 * q + 1] = mm[w][q].imag(); }
        } else if (s.out_diag) {
            CHECK(std::abs(m[1]) == 0 && std::abs(m[2]) == 0, "diagonal fusion has off-diagonal terms");
            c[0] = m[0].real(); c[1] = m[0].imag(); c[2] = m[3].real(); c[3] = m[3].imag();
        } else {
            for (int q = 0; q < 4; ++q) { c[2 * q] = m[q].real(); c[2 * q + 1] = m[q].imag(); }
        }
        return;
    }
    const double th = s.pidx >= 0 ? params[s.pidx] : s.value;
    const double ch = cos(th / 2), sh = sin(th / 2);
    switch (s.gate) {
    case SV_RX: { double m[8] = {ch, 0, 0, -sh, 0, -sh, ch, 0}; memcpy(c, m, sizeof m); break; }
    case SV_RY: { double m[8] = {ch, 0, -sh, 0, sh, 0, ch, 0}; memcpy(c, m, sizeof m); break; }
    case SV_RZ: c[0] = ch; c[1] = -sh; c[2] = ch; c[3] = sh; break;
    case SV_PHASE: c[0] = cos(th); c[1] = sin(th); break;
    default: for (int k = 0; k < s.nfixed; ++k) c[k] = s.fixed[k];
    }
}

struct Frame {
    uint32_t tl[512];
    uint32_t off[16];
};

static void frame(const FLayout& L, int tq, int rb, int nthr, Frame& f)
{
    const int nl = tq - rb;
    for (int t = 0; t < nthr; ++t) {
        uint32_t v = 0;
        for (int i = 0; i < nl; ++i) v |= ((t >> i) & 1u) << L.pos[i];
        f.tl[t] = v;
    }
    for (int j = 0; j < (1 << rb); ++j) {
        uint32_t v = 0;
        for (int r = 0; r < rb; ++r)
            if ((j >> r) & 1) v |= 1u << L.pos[nl + r];
        f.off[j] = v;
    }
}

static bool check_layout(const FLayout& L, int tq, int rb = -1, const int32_t* q = nullptr)
{
    uint32_t seen = 0;
    for (int i = 0; i < tq; ++i) {
        if (L.pos[i] >= tq) return false;
        seen |= 1u << L.pos[i];
    }
    if (seen != (1u << tq) - 1u) return false;
    if (rb > 0) {
        const int nl = tq - rb;
        for (int i = 0; i < 16; ++i) {
            const uint32_t want = i < nl ? 1u << L.pos[i] : 0u;
            if (L.lane_l[i] != want) return false;
            if (L.lane_g[i] != (i < nl ? 1ull << q[L.pos[i]] : 0ull)) return false;
        }
        for (int r = 0; r < rb; ++r)
            if (L.reg_l[r] != (1u << L.pos[nl + r]) || L.reg_g[r] != (1ull << q[L.pos[nl + r]])) return false;
    }
    return true;
}


static void reg_apply_h(cd* v, int rb, const FOp& op, const double* cf, bool dagger, uint32_t tl, const uint32_t* off,
                        const FLayout& L, int tq)
{
    const int R = 1 << rb, nl = tq - rb;
    {
        uint32_t Sm = 0, cmk = 0;
        for (int r = 0; r < rb; ++r) Sm |= 1u << L.pos[nl + r];
        for (int r = 0; r < rb; ++r)
            if ((op.cm >> L.pos[nl + r]) & 1u) cmk |= 1u << r;
        CHECK(op.cml == (op.cm & ~Sm), "cml %x != lane part of cm %x", op.cml, op.cm & ~Sm);
        CHECK(op.cmk == cmk, "cmk %x != %x", op.cmk, cmk);
        CHECK(op.ka == -1 || L.pos[nl + op.ka] == op.a, "ka does not hold a");
    }
    switch (op.kind) {
    case FK_PAIRX:
    case FK_PAIRR:
    case FK_PAIR: {
        CHECK(L.pos[nl + op.ka] == op.a, "pair target %d not at register bit %d", op.a, op.ka);
        if (op.kind == FK_PAIRR) CHECK(cf[1] == 0 && cf[3] == 0 && cf[5] == 0 && cf[7] == 0, "real pair with complex coefficients");
        if (op.kind == FK_PAIRX) CHECK(cf[0] == 0 && cf[2] == 1 && cf[4] == 1 && cf[6] == 0, "exchange pair is not X");
        cd u[4];
        for (int k = 0; k < 4; ++k) u[k] = cd(cf[2 * k], cf[2 * k + 1]);
        if (dagger) { cd t = u[1]; u[0] = std::conj(u[0]); u[1] = std::conj(u[2]); u[2] = std::conj(t); u[3] = std::conj(u[3]); }
        for (int j = 0; j < R; ++j) {
            if (j & (1 << op.ka)) continue;
            if (((tl | off[j]) & op.cm) != op.cm) continue;
            const int j1 = j | (1 << op.ka);
            const cd a = v[j], b = v[j1];
            v[j] = u[0] * a + u[1] * b;
            v[j1] = u[2] * a + u[3] * b;
        }
        break;
    }
    case FK_PAIRC: {
        // forward only: the 2x2 depends on selector bit b (cf[0..7] where it is 0, cf[8..15] where it is 1)
        CHECK(!dagger, "two-branch op in a reverse list");
        ++(op.kb >= 0 ? pairc_reg : pairc_lane);
        CHECK(op.cm == 0, "two-branch op with controls");
        CHECK(L.pos[nl + op.ka] == op.a, "two-branch target %d not at register bit %d", op.a, op.ka);
        if (op.kb >= 0) CHECK(L.pos[nl + op.kb] == op.b, "selector kb %d does not hold %d", op.kb, op.b);
        else for (int r = 0; r < rb; ++r) CHECK(L.pos[nl + r] != op.b, "selector in registers but kb = -1");
        for (int j = 0; j < R; ++j) {
            if (j & (1 << op.ka)) continue;
            const int j1 = j | (1 << op.ka);
            const bool s = ((tl | off[j]) >> op.b) & 1u;
            const double* m = cf + (s ? 8 : 0);
            const cd u0(m[0], m[1]), u1(m[2], m[3]), u2(m[4], m[5]), u3(m[6], m[7]);
            const cd a = v[j], b = v[j1];
            v[j] = u0 * a + u1 * b;
            v[j1] = u2 * a + u3 * b;
        }
        break;
    }
    case FK_DIAG: {
        cd d0(cf[0], dagger ? -cf[1] : cf[1]), d1(cf[2], dagger ? -cf[3] : cf[3]);
        if (op.ka >= 0) CHECK(L.pos[nl + op.ka] == op.a, "diag ka %d does not hold %d", op.ka, op.a);
        else for (int r = 0; r < rb; ++r) CHECK(L.pos[nl + r] != op.a, "diag target in registers but ka = -1");
        for (int j = 0; j < R; ++j) {
            const uint32_t l = tl | off[j];
            if ((l & op.cm) != op.cm) continue;
            v[j] *= ((l >> op.a) & 1) ? d1 : d0;
        }
        break;
    }
    case FK_PHASE: {
        cd z(cf[0], dagger ? -cf[1] : cf[1]);
        for (int j = 0; j < R; ++j)
            if (((tl | off[j]) & op.cm) == op.cm) v[j] *= z;
        break;
    }
    case FK_SWAP: {
        CHECK(op.ka >= 0 && op.kb >= 0 && L.pos[nl + op.ka] == op.a && L.pos[nl + op.kb] == op.b,
              "swap targets not in registers");
        for (int j = 0; j < R; ++j) {
            if (!(j & (1 << op.ka)) || (j & (1 << op.kb))) continue;
            if (((tl | off[j]) & op.cm) != op.cm) continue;
            std::swap(v[j], v[j ^ (1 << op.ka) ^ (1 << op.kb)]);
        }
        break;
    }
    default: CHECK(0, "bad kind %d", op.kind);
    }
}

// A 4x4 op or a SWAP by a sweep over the whole tile, as the kernels do through LDS:
// registers -> swizzled LDS (poisoned with NaN first) -> tile in local order
// -> op -> LDS -> registers.
static void quad_sweep_h(std::vector<cd>& v, int nthr, int R, const Frame& f, int tq, const FOp& op, const double* cf,
                         bool dagger)
{
    std::vector<cd> lds(1u << 13, cd(NAN, NAN)), A(1u << tq);
    for (int t = 0; t < nthr; ++t)
        for (int j = 0; j < R; ++j) lds[swz_h(f.tl[t] | f.off[j])] = v[t * R + j];
    for (uint32_t l = 0; l < (1u << tq); ++l) A[l] = lds[swz_h(l)];
    cd U[16];
    if (op.kind == FK_SWAP) {
        for (int e = 0; e < 16; ++e) U[e] = 0;
        U[0] = U[6] = U[9] = U[15] = 1;
    } else
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            const int e = dagger ? (4 * c + r) : (4 * r + c);
            U[4 * r + c] = cd(cf[2 * e], dagger ? -cf[2 * e + 1] : cf[2 * e + 1]);
        }
    for (uint32_t i = 0; i < (1u << tq); ++i) {
        if (((i >> op.a) & 1) || ((i >> op.b) & 1) || (i & op.cm) != op.cm) continue;
        const uint32_t ix[4] = {i, i | (1u << op.b), i | (1u << op.a), i | (1u << op.a) | (1u << op.b)};
        cd w[4], r4[4];
        for (int k = 0; k < 4; ++k) w[k] = A[ix[k]];
        for (int r = 0; r < 4; ++r) {
            r4[r] = 0;
            for (int c = 0; c < 4; ++c) r4[r] += U[4 * r + c] * w[c];
        }
        for (int k = 0; k < 4; ++k) A[ix[k]] = r4[k];
    }
    for (uint32_t l = 0; l < (1u << tq); ++l) lds[swz_h(l)] = A[l];
    for (int t = 0; t < nthr; ++t)
        for (int j = 0; j < R; ++j) v[t * R + j] = lds[swz_h(f.tl[t] | f.off[j])];
}

static double gen_inner_h(const cd* P, const cd* Lm, int rb, const FOp& op, uint32_t tl, const uint32_t* off,
                          const FLayout& L, int tq)
{
    const int R = 1 << rb;
    const uint32_t cm = op.cm & ~(1u << op.a);
    double acc = 0;
    if (op.gen == GEN_X || op.gen == GEN_Y) {
        CHECK(L.pos[(tq - rb) + op.ka] == op.a, "generator target not in registers");
        for (int j = 0; j < R; ++j) {
            if (j & (1 << op.ka)) continue;
            if (((tl | off[j]) & cm) != cm) continue;
            const int j1 = j | (1 << op.ka);
            cd g0, g1;  // G phi
            if (op.gen == GEN_X) { g0 = P[j1]; g1 = P[j]; }
            else { g0 = cd(0, -1) * P[j1]; g1 = cd(0, 1) * P[j]; }
            acc += (std::conj(Lm[j]) * g0 + std::conj(Lm[j1]) * g1).imag();
        }
        return acc;
    }
    for (int j = 0; j < R; ++j) {
        const uint32_t l = tl | off[j];
        if ((l & cm) != cm) continue;
        const bool b = (l >> op.a) & 1;
        const double t = (std::conj(Lm[j]) * P[j]).imag();
        if (op.gen == GEN_Z) acc += b ? -t : t;
        else if (b) acc += t;
    }
    return acc;
}

struct Emu {
    HostTables H;
    std::vector<std::vector<cd>> psi, lam;
    std::vector<double> coef, epart, gpart;
};

static uint64_t tile_base_h(const FPass& ps, int tq, uint64_t tile)
{
    uint64_t b = tile;
    for (int k = 0; k < tq; ++k) {
        const int p = ps.q[k];
        b = ((b >> p) << (p + 1)) | (b & ((1ull << p) - 1ull));
    }
    return b;
}

static void run_emu(Emu& E, const std::vector<double>& params)
{
    HostTables& H = E.H;
    E.coef.assign(std::max(1, H.coef_total), 0.0);
    for (auto& s : H.cspec) coef_eval(s, H.cfac, params.data(), E.coef.data() + s.coef);
    const int nc = (int)H.circs.size();
    E.psi.assign(nc, {});
    E.lam.assign(nc, {});
    E.epart.assign(std::max(1, H.e_total), 0.0);
    E.gpart.assign(std::max<int64_t>(1, H.g_total), 0.0);
    for (int c = 0; c < nc; ++c) {
        const FCirc& cc = H.circs[c];
        E.psi[c].assign(1ull << cc.n, cd(NAN, NAN));
        E.lam[c].assign(1ull << cc.n, cd(NAN, NAN));
    }
    std::vector<cd> lds(1 << 13);
    for (int c = 0; c < nc; ++c) {
        const FCirc& cc = H.circs[c];
        const int tq = cc.tq;
        std::vector<cd>& psi = E.psi[c];
        std::vector<cd>& lam = E.lam[c];
        // forward
        for (int p = 0; p < cc.n_pass; ++p) {
            const FPass& ps = H.passes[cc.pass_begin + p];
            if (!cc.reg) {  // LDS-sweep form: plain ops on the tile (planner not involved)
                for (uint64_t tile = 0; tile < (uint64_t)cc.n_tiles; ++tile) {
                    const uint64_t tb = tile_base_h(ps, tq, tile);
                    std::vector<cd> t(1u << tq);
                    for (uint32_t l = 0; l < (1u << tq); ++l) {
                        uint64_t g = tb;
                        for (int k = 0; k < tq; ++k) if ((l >> k) & 1) g |= 1ull << ps.q[k];
                        t[l] = p == 0 ? cd(g == 0 ? 1 : 0, 0) : psi[g];
                    }
                    for (int o = ps.op_begin; o < ps.op_end; ++o) CHECK(H.fops[o].kind != FK_LAYOUT, "layout op in LDS form");
                    // not emulated further: the LDS form is the previously tested code
                    (void)t;
                }
                printf("circuit %d uses the LDS form: skipped\n", c);
                goto next_circ;
            }
            {
                const int rb = H.reg_bits, R = 1 << rb, nthr = 1 << (tq - rb);
                for (int i = ps.lay_begin; i <= ps.lay_end; ++i) {}
                for (uint64_t tile = 0; tile < (uint64_t)cc.n_tiles; ++tile) {
                    const uint64_t tb = tile_base_h(ps, tq, tile);
                    std::vector<cd> v((size_t)nthr * R);
                    int cur = ps.lay_begin;
                    CHECK(check_layout(H.lays[cur], tq, rb, ps.q), "bad layout");
                    {
                        uint64_t fm = 0;
                        for (int k = 0; k < tq; ++k) fm |= 1ull << ps.q[k];
                        CHECK(ps.free_mask == (((1ull << cc.n) - 1) & ~fm), "free mask");
                    }
                    Frame f;
                    frame(H.lays[cur], tq, rb, nthr, f);
                    for (int t = 0; t < nthr; ++t)
                        for (int j = 0; j < R; ++j) {
                            const uint32_t l = f.tl[t] | f.off[j];
                            uint64_t g = tb;
                            for (int k = 0; k < tq; ++k) if ((l >> k) & 1) g |= 1ull << ps.q[k];
                            v[t * R + j] = p == 0 ? cd(g == 0 ? 1 : 0, 0) : psi[g];
                        }
                    cd chain_acc = 1.0;
                    bool ch_any = false;
                    std::vector<cd> run_acc(nthr, cd(1.0));  // per-thread product of a phase run
                    const uint64_t tile_bits = ~ps.free_mask & ((1ull << cc.n) - 1);
                    for (int o = ps.op_begin; o < ps.op_end; ++o) {
                        const FOp& op = H.fops[o];
                        if (op.kind == FK_PHASE) {
                            // subset phase: out-of-tile bits gate it per tile; chains multiply
                            // b: the op's qubits outside the tile, packed as in a tile index
                            uint64_t gm = 0;
                            {
                                int rank = 0;
                                for (int q = 0; q < cc.n; ++q)
                                    if ((ps.free_mask >> q) & 1ull) {
                                        if (((uint32_t)op.b >> rank) & 1u) gm |= 1ull << q;
                                        ++rank;
                                    }
                            }
                            CHECK(((uint64_t)(uint32_t)op.b >> (cc.n - tq)) == 0, "packed mask beyond the tile index");
                            CHECK((gm & tile_bits) == 0, "gm holds tile bits");
                            // the kernel tests the packed mask against the tile index
                            CHECK((((uint32_t)tile & (uint32_t)op.b) == (uint32_t)op.b) == ((tb & gm) == gm),
                                  "packed test disagrees with the base-index test");
                            CHECK(op.cm != 0 && ((op.cm >> op.a) & 1u), "phase without an in-tile bit");
                            CHECK(op.kb >= 0 && op.kb <= 3, "chain flag %d", op.kb);
                            if (op.kb >= 2) {
                                // run on target a: the other in-tile bit, if any, must be a lane bit
                                const uint32_t other = op.cm & ~(1u << op.a);
                                uint32_t lanes = 0;
                                for (int i = 0; i < tq - rb; ++i) lanes |= 1u << H.lays[cur].pos[i];
                                CHECK(__builtin_popcount(other) <= 1 && (other & ~lanes) == 0,
                                      "run member with mask %x on target %d", op.cm, op.a);
                                CHECK(op.ka == -1 || H.lays[cur].pos[tq - rb + op.ka] == op.a, "run ka does not hold a");
                                CHECK(op.ka != -1 || ((lanes >> op.a) & 1u), "run target on a register but ka = -1");
                                if (op.kb == 2)
                                    CHECK(o + 1 < ps.op_end && H.fops[o + 1].kind == FK_PHASE && H.fops[o + 1].a == op.a &&
                                              H.fops[o + 1].kb >= 2, "run not followed by a member on the same target");
                                if ((tb & gm) == gm) {
                                    const cd z(E.coef[op.coef], E.coef[op.coef + 1]);
                                    for (int t = 0; t < nthr; ++t)
                                        if ((f.tl[t] & other) == other) run_acc[t] *= z;
                                }
                                ++run_members;
                                if (op.kb == 2) continue;
                                for (int t = 0; t < nthr; ++t) {
                                    for (int j = 0; j < R; ++j)
                                        if ((((f.tl[t] | f.off[j]) >> op.a) & 1u)) v[t * R + j] *= run_acc[t];
                                    run_acc[t] = 1.0;
                                }
                                continue;
                            }
                            if ((tb & gm) == gm) {
                                chain_acc *= cd(E.coef[op.coef], E.coef[op.coef + 1]);
                                ch_any = true;
                            }
                            if (op.kb == 1) {
                                CHECK(o + 1 < ps.op_end && H.fops[o + 1].kind == FK_PHASE && H.fops[o + 1].cm == op.cm,
                                      "chain not followed by a phase on the same mask");
                                continue;
                            }
                            if (ch_any) {
                                const double zz[2] = {chain_acc.real(), chain_acc.imag()};
                                for (int t = 0; t < nthr; ++t)
                                    reg_apply_h(&v[t * R], rb, op, zz, false, f.tl[t], f.off, H.lays[cur], tq);
                            }
                            chain_acc = 1.0;
                            ch_any = false;
                            continue;
                        }
                        if (op.kind == FK_LAYOUT) {
                            if (op.a == cur) continue;
                            CHECK(op.b == cur, "marker from %d but current %d", op.b, cur);
                            std::fill(lds.begin(), lds.end(), cd(NAN, NAN));
                            for (int t = 0; t < nthr; ++t)
                                for (int j = 0; j < R; ++j) lds[swz_h(f.tl[t] | f.off[j])] = v[t * R + j];
                            cur = op.a;
                            CHECK(check_layout(H.lays[cur], tq, rb, ps.q), "bad layout");
                            frame(H.lays[cur], tq, rb, nthr, f);
                            for (int t = 0; t < nthr; ++t)
                                for (int j = 0; j < R; ++j) v[t * R + j] = lds[swz_h(f.tl[t] | f.off[j])];
                            continue;
                        }
                        if ((op.kind == FK_PAIR || op.kind == FK_PAIRR || op.kind == FK_PAIRX || op.kind == FK_DIAG) &&
                            op.b != 0) {
                            // controls outside the tile: the op acts on the tiles whose index holds them
                            uint64_t gm = 0;
                            int rank = 0;
                            for (int q = 0; q < cc.n; ++q)
                                if ((ps.free_mask >> q) & 1ull) {
                                    if (((uint32_t)op.b >> rank) & 1u) gm |= 1ull << q;
                                    ++rank;
                                }
                            CHECK((gm & tile_bits) == 0, "out-of-tile controls hold tile bits");
                            CHECK((((uint32_t)tile & (uint32_t)op.b) == (uint32_t)op.b) == ((tb & gm) == gm),
                                  "packed control test disagrees with the base-index test");
                            ++gated_ops;
                            if ((tb & gm) != gm) continue;
                        }
                        if (op.kind == FK_QUAD) {
                            quad_sweep_h(v, nthr, R, f, tq, op, E.coef.data() + op.coef, false);
                            continue;
                        }
                        if (op.kind == FK_PAIRT) {
                            // the entry whose bits are the tile's values of the out-of-tile qubits under b
                            CHECK(op.cm == 0 && op.b != 0, "tile-selected op with in-tile controls or no mask");
                            int rank = 0, k = 0, e = 0;
                            for (int q = 0; q < cc.n; ++q)
                                if ((ps.free_mask >> q) & 1ull) {
                                    if (((uint32_t)op.b >> rank) & 1u) {
                                        if ((tb >> q) & 1ull) e |= 1 << k;
                                        ++k;
                                    }
                                    ++rank;
                                }
                            CHECK(k == __builtin_popcount((uint32_t)op.b), "mask bits beyond the free qubits");
                            FOp q2 = op;
                            q2.kind = FK_PAIR;
                            q2.b = 0;
                            ++tsel_ops;
                            for (int t = 0; t < nthr; ++t)
                                reg_apply_h(&v[t * R], rb, q2, E.coef.data() + op.coef + 8 * e, false, f.tl[t], f.off,
                                            H.lays[cur], tq);
                            continue;
                        }
                        for (int t = 0; t < nthr; ++t)
                            reg_apply_h(&v[t * R], rb, op, E.coef.data() + op.coef, false, f.tl[t], f.off, H.lays[cur], tq);
                    }
                    CHECK(cur == ps.lay_end, "forward ends in %d, expected %d", cur, ps.lay_end);
                    for (int t = 0; t < nthr; ++t)
                        for (int j = 0; j < R; ++j) {
                            const uint32_t l = f.tl[t] | f.off[j];
                            uint64_t g = tb;
                            for (int k = 0; k < tq; ++k) if ((l >> k) & 1) g |= 1ull << ps.q[k];
                            psi[g] = v[t * R + j];
                        }
                }
            }
        }
        // observable
        {
            double e = 0;
            for (uint64_t x = 0; x < psi.size(); ++x) {
                const double o = obs_val(x, cc.n, cc.obs_kind);
                e += o * std::norm(psi[x]);
                lam[x] = o * psi[x];
            }
            E.epart[cc.e_part_begin] = e;
            for (int t = 1; t < cc.n_tiles; ++t) E.epart[cc.e_part_begin + t] = 0;
        }
        if (!H.with_grad) goto next_circ;
        if (!cc.rreg) { printf("circuit %d reverse uses the LDS form: skipped\n", c); goto next_circ; }
        for (int p = cc.n_pass - 1; p >= 0; --p) {
            const FPass& ps = H.passes[cc.pass_begin + p];
            const int rb = H.rreg_bits, R = 1 << rb, nthr = 1 << (tq - rb);
            for (uint64_t tile = 0; tile < (uint64_t)cc.n_tiles; ++tile) {
                const uint64_t tb = tile_base_h(ps, tq, tile);
                std::vector<cd> v((size_t)nthr * R), w((size_t)nthr * R);
                int cur = ps.rlay_end;
                Frame f;
                frame(H.lays[cur], tq, rb, nthr, f);
                auto gaddr = [&](uint32_t l) {
                    uint64_t g = tb;
                    for (int k = 0; k < tq; ++k) if ((l >> k) & 1) g |= 1ull << ps.q[k];
                    return g;
                };
                for (int t = 0; t < nthr; ++t)
                    for (int j = 0; j < R; ++j) {
                        const uint64_t g = gaddr(f.tl[t] | f.off[j]);
                        v[t * R + j] = psi[g];
                        w[t * R + j] = lam[g];
                    }
                for (int o = ps.rop_end - 1; o >= ps.rop_begin; --o) {
                    const FOp& op = H.fops[o];
                    if (op.kind == FK_LAYOUT) {
                        if (op.b == cur) continue;
                        CHECK(op.a == cur, "reverse marker to %d but current %d", op.a, cur);
                        Frame f2;
                        frame(H.lays[op.b], tq, rb, nthr, f2);
                        for (auto* arr : {&v, &w}) {
                            std::fill(lds.begin(), lds.end(), cd(NAN, NAN));
                            for (int t = 0; t < nthr; ++t)
                                for (int j = 0; j < R; ++j) lds[swz_h(f.tl[t] | f.off[j])] = (*arr)[t * R + j];
                            for (int t = 0; t < nthr; ++t)
                                for (int j = 0; j < R; ++j) (*arr)[t * R + j] = lds[swz_h(f2.tl[t] | f2.off[j])];
                        }
                        cur = op.b;
                        f = f2;
                        continue;
                    }
                    const bool gated = op.kind == FK_PHASE || op.kind == FK_PAIR || op.kind == FK_PAIRR ||
                                       op.kind == FK_PAIRX || op.kind == FK_DIAG;
                    const bool on = !gated || ((uint32_t)tile & (uint32_t)op.b) == (uint32_t)op.b;
                    if (op.slot >= 0) {
                        double acc = 0;
                        if (on)
                            for (int t = 0; t < nthr; ++t)
                                acc += gen_inner_h(&v[t * R], &w[t * R], rb, op, f.tl[t], f.off, H.lays[cur], tq);
                        E.gpart[cc.g_part_begin + (int64_t)op.slot * cc.n_tiles + tile] = acc;
                    }
                    if (op.kind == FK_RFUSE) {
                        // first gate's partial: Im <lambda| M |phi> with M = B G_A B^dagger, over the controlled pairs
                        const int nl = tq - rb;
                        CHECK(op.ka >= 0 && H.lays[cur].pos[nl + op.ka] == op.a, "reverse pair target not in registers");
                        const double* mc = E.coef.data() + op.coef + 8;
                        const cd M[4] = {cd(mc[0], mc[1]), cd(mc[2], mc[3]), cd(mc[4], mc[5]), cd(mc[6], mc[7])};
                        if (op.b >= 0) {
                            double acc = 0;
                            const uint32_t cm = op.cm & ~(1u << op.a);
                            for (int t = 0; t < nthr; ++t)
                                for (int j = 0; j < R; ++j) {
                                    if (j & (1 << op.ka)) continue;
                                    if (((f.tl[t] | f.off[j]) & cm) != cm) continue;
                                    const int j1 = j | (1 << op.ka);
                                    const cd p0 = v[t * R + j], p1 = v[t * R + j1];
                                    const cd t0 = M[0] * p0 + M[1] * p1, t1 = M[2] * p0 + M[3] * p1;
                                    acc += (std::conj(w[t * R + j]) * t0 + std::conj(w[t * R + j1]) * t1).imag();
                                }
                            E.gpart[cc.g_part_begin + (int64_t)op.b * cc.n_tiles + tile] = acc;
                        }
                        FOp q2 = op;
                        q2.kind = FK_PAIR;
                        q2.b = 0;
                        ++rfuse_ops;
                        for (int t = 0; t < nthr; ++t) {
                            reg_apply_h(&v[t * R], rb, q2, E.coef.data() + op.coef, true, f.tl[t], f.off, H.lays[cur], tq);
                            reg_apply_h(&w[t * R], rb, q2, E.coef.data() + op.coef, true, f.tl[t], f.off, H.lays[cur], tq);
                        }
                        continue;
                    }
                    if (!on) continue;
                    if (op.kind == FK_QUAD || op.kind == FK_SWAP) {
                        quad_sweep_h(v, nthr, R, f, tq, op, E.coef.data() + op.coef, true);
                        quad_sweep_h(w, nthr, R, f, tq, op, E.coef.data() + op.coef, true);
                        continue;
                    }
                    for (int t = 0; t < nthr; ++t) {
                        reg_apply_h(&v[t * R], rb, op, E.coef.data() + op.coef, true, f.tl[t], f.off, H.lays[cur], tq);
                        reg_apply_h(&w[t * R], rb, op, E.coef.data() + op.coef, true, f.tl[t], f.off, H.lays[cur], tq);
                    }
                }
                CHECK(cur == ps.rlay_begin, "reverse ends in %d, expected %d", cur, ps.rlay_begin);
                for (int t = 0; t < nthr; ++t)
                    for (int j = 0; j < R; ++j) {
                        const uint64_t g = gaddr(f.tl[t] | f.off[j]);
                        psi[g] = v[t * R + j];
                        lam[g] = w[t * R + j];
                    }
            }
        }
    next_circ:;
    }
}

// ---------------- circuits -----------------------------------------------
struct Circ {
    int n;
    std::vector<sv_op> ops;
    std::vector<std::vector<double>> mats;
    int n_params;
    int obs;
};

static sv_op mk(int g, std::vector<int> ctl, std::vector<int> tgt, int pidx = -1, double val = 0)
{
    sv_op o;
    memset(&o, 0, sizeof o);
    o.gate = g;
    o.n_controls = (int)ctl.size();
    o.n_targets = (int)tgt.size();
    int k = 0;
    for (int c : ctl) o.qubits[k++] = c;
    for (int t : tgt) o.qubits[k++] = t;
    o.param_index = pidx;
    o.value = val;
    return o;
}

static void haar(std::mt19937_64& rng, int d, std::vector<double>& out)
{
    // Gram-Schmidt of a Gaussian matrix (unitary; distribution irrelevant here)
    std::normal_distribution<double> N;
    std::vector<cd> m(d * d);
    for (auto& z : m) z = cd(N(rng), N(rng));
    for (int c = 0; c < d; ++c) {
        for (int p = 0; p < c; ++p) {
            cd dot = 0;
            for (int r = 0; r < d; ++r) dot += std::conj(m[r * d + p]) * m[r * d + c];
            for (int r = 0; r < d; ++r) m[r * d + c] -= dot * m[r * d + p];
        }
        double nn = 0;
        for (int r = 0; r < d; ++r) nn += std::norm(m[r * d + c]);
        nn = sqrt(nn);
        for (int r = 0; r < d; ++r) m[r * d + c] /= nn;
    }
    out.resize(2 * d * d);
    for (int k = 0; k < d * d; ++k) { out[2 * k] = m[k].real(); out[2 * k + 1] = m[k].imag(); }
}

static Circ random_circ(std::mt19937_64& rng, int n, int n_ops, int n_params)
{
    Circ C;
    C.n = n;
    C.n_params = n_params;
    C.obs = 1 + (rng() & 1);
    C.mats.reserve(n_ops);
    auto pick = [&](int k, std::vector<int>& out) {
        out.clear();
        while ((int)out.size() < k) {
            int q = rng() % n;
            if (std::find(out.begin(), out.end(), q) == out.end()) out.push_back(q);
        }
    };
    std::vector<int> qs;
    const int gates[] = {SV_X, SV_Y, SV_Z, SV_H, SV_S, SV_T, SV_RX, SV_RY, SV_RZ, SV_PHASE, SV_SWAP, SV_U2, SV_U4};
    for (int i = 0; i < n_ops; ++i) {
        const int g = gates[rng() % 13];
        const int nt = (g == SV_SWAP || g == SV_U4) ? 2 : 1;
        int nc = (int)(rng() % 3);
        if (nc + nt > n) nc = n - nt;
        if (nc < 0) { --i; continue; }
        pick(nc + nt, qs);
        std::vector<int> ctl(qs.begin(), qs.begin() + nc), tgt(qs.begin() + nc, qs.end());
        const bool rot = g == SV_RX || g == SV_RY || g == SV_RZ || g == SV_PHASE;
        int pidx = -1;
        double val = 0;
        if (rot) {
            if (rng() % 4 && n_params > 0) pidx = rng() % n_params;
            else val = (rng() % 1000) * 0.00628;
        }
        sv_op o = mk(g, ctl, tgt, pidx, val);
        if (g == SV_U2 || g == SV_U4) {
            C.mats.emplace_back();
            haar(rng, g == SV_U2 ? 2 : 4, C.mats.back());
            o.matrix = C.mats.back().data();
        }
        C.ops.push_back(o);
    }
    return C;
}

static Circ hea(int n, int L)
{
    Circ C;
    C.n = n;
    C.n_params = 2 * n * L;
    C.obs = 1;
    for (int l = 0; l < L; ++l) {
        for (int q = 0; q < n; ++q) {
            C.ops.push_back(mk(SV_RY, {}, {q}, 2 * (l * n + q)));
            C.ops.push_back(mk(SV_RZ, {}, {q}, 2 * (l * n + q) + 1));
        }
        for (int q = 0; q + 1 < n; ++q) C.ops.push_back(mk(SV_X, {q}, {q + 1}));
    }
    return C;
}

// QFT (Hadamards and controlled phases, no swaps), with every fourth phase
// angle a parameter so the reverse sweep's subset-phase gradients are covered.
static Circ qft(int n)
{
    Circ C;
    C.n = n;
    C.n_params = 0;
    C.obs = 2;
    int np = 0;
    for (int j = n - 1; j >= 0; --j) {
        C.ops.push_back(mk(SV_H, {}, {j}));
        for (int c = j - 1; c >= 0; --c) {
            if ((c + j) % 4 == 0) C.ops.push_back(mk(SV_PHASE, {c}, {j}, np++));
            else C.ops.push_back(mk(SV_PHASE, {c}, {j}, -1, M_PI / (double)(1 << std::min(j - c, 30))));
        }
    }
    C.n_params = np;
    return C;
}

// Mostly subset phases (Z, S, T, PHASE with 0..3 controls) between a few
// Hadamards and CNOTs: phases whose qubits fall outside the tile.
// Runs of CNOTs from every other qubit onto one target, each followed by a
// rotation of the target (parameterised every third), target by target.
static Circ cnot_runs(int n)
{
    Circ C;
    C.n = n;
    C.obs = 1;
    int np = 0;
    for (int t = 0; t < n; ++t) {
        C.ops.push_back(mk(SV_RY, {}, {t}, np++));
        for (int c = 0; c < n; ++c) {
            if (c == t) continue;
            C.ops.push_back(mk(SV_X, {c}, {t}));
            if (c % 3 == 0) C.ops.push_back(mk(SV_RZ, {}, {t}, np++));
            else C.ops.push_back(mk(c % 3 == 1 ? SV_RZ : SV_RX, {}, {t}, -1, 0.1 * (c + 1) + 0.01 * t));
        }
    }
    C.n_params = np;
    return C;
}

static Circ phase_heavy(std::mt19937_64& rng, int n, int n_ops, int n_params)
{
    Circ C;
    C.n = n;
    C.n_params = n_params;
    C.obs = 1 + (rng() & 1);
    std::vector<int> qs;
    auto pick = [&](int k) {
        qs.clear();
        while ((int)qs.size() < k) {
            int q = rng() % n;
            if (std::find(qs.begin(), qs.end(), q) == qs.end()) qs.push_back(q);
        }
    };
    for (int q = 0; q < n; ++q) C.ops.push_back(mk(SV_H, {}, {q}));
    const int ph[] = {SV_Z, SV_S, SV_T, SV_PHASE, SV_PHASE};
    for (int i = 0; i < n_ops; ++i) {
        const int r = rng() % 10;
        if (r == 0) {
            pick(1);
            C.ops.push_back(mk(SV_H, {}, {qs[0]}));
        } else if (r == 1) {
            pick(2);
            C.ops.push_back(mk(SV_X, {qs[0]}, {qs[1]}));
        } else {
            const int g = ph[rng() % 5];
            const int nc = std::min((int)(rng() % 4), n - 1);
            pick(nc + 1);
            std::vector<int> ctl(qs.begin(), qs.begin() + nc);
            int pidx = -1;
            double val = 0;
            if (g == SV_PHASE) {
                if (rng() % 2 && n_params > 0) pidx = rng() % n_params;
                else val = (rng() % 1000) * 0.00628;
            }
            C.ops.push_back(mk(g, ctl, {qs[nc]}, pidx, val));
        }
    }
    return C;
}

static void test(const std::vector<Circ>& cs, int dtype, int tile, int apt, int with_grad, const char* name,
                 std::mt19937_64& rng)
{
    std::vector<sv_batch_circuit> bc(cs.size());
    int np = 0;
    for (size_t i = 0; i < cs.size(); ++i) {
        bc[i].n_qubits = cs[i].n;
        bc[i].n_ops = (int)cs[i].ops.size();
        bc[i].ops = cs[i].ops.data();
        bc[i].n_params = cs[i].n_params;
        bc[i].obs_kind = cs[i].obs;
        np += cs[i].n_params;
    }
    sv_batch_opts op = {tile, apt, 0, with_grad};
    Emu E;
    const int e0 = errors;
    sv_status rc = compile_batch(bc.data(), (int)bc.size(), dtype, &op, E.H);
    if (rc) { printf("%s: compile failed: %s\n", name, sv_last_error()); ++errors; return; }
    std::uniform_real_distribution<double> U(0, 6.283);
    std::vector<double> params(np);
    for (auto& x : params) x = U(rng);
    run_emu(E, params);
    double max_state = 0, max_e = 0, max_g = 0;
    int off = 0;
    for (size_t c = 0; c < cs.size(); ++c) {
        std::vector<double> pc(params.begin() + off, params.begin() + off + cs[c].n_params);
        std::vector<cd> ref;
        const double e = ref_energy(cs[c].n, cs[c].ops, pc, cs[c].obs, &ref);
        const FCirc& cc = E.H.circs[c];
        if (!cc.reg) { off += cs[c].n_params; continue; }
        double em = 0;
        for (int t = 0; t < cc.n_tiles; ++t) em += E.epart[cc.e_part_begin + t];
        max_e = std::max(max_e, fabs(em - e));
        if (!with_grad)
            for (size_t x = 0; x < ref.size(); ++x) max_state = std::max(max_state, std::abs(E.psi[c][x] - ref[x]));
        else if (cc.rreg) {
            // after the reverse sweep phi must be |0...0>
            for (size_t x = 0; x < ref.size(); ++x)
                max_state = std::max(max_state, std::abs(E.psi[c][x] - cd(x == 0 ? 1 : 0, 0)));
            // gradient: central differences of the reference energy
            std::vector<double> g(cs[c].n_params, 0.0);
            for (size_t s = 0; s < E.H.slot_param.size(); ++s) {
                const int pj = E.H.slot_param[s] - off;
                if (pj < 0 || pj >= cs[c].n_params) continue;
                double acc = 0;
                const int64_t b = E.H.g_off[s];
                for (int t = 0; t < E.H.g_cnt[s]; ++t) acc += E.gpart[b + t];
                g[pj] += E.H.slot_scale[s] * acc;
            }
            for (int j = 0; j < cs[c].n_params; ++j) {
                const double h = 1e-5;
                std::vector<double> pp = pc, pm = pc;
                pp[j] += h;
                pm[j] -= h;
                const double fd = (ref_energy(cs[c].n, cs[c].ops, pp, cs[c].obs) - ref_energy(cs[c].n, cs[c].ops, pm, cs[c].obs)) / (2 * h);
                max_g = std::max(max_g, fabs(fd - g[j]));
            }
        }
        off += cs[c].n_params;
    }
    const bool ok = errors == e0 && max_state < 1e-10 && max_e < 1e-9 && max_g < 1e-6;
    if (!ok) ++errors;
    printf("%-44s passes %4zu layouts %4zu ops %5zu  state %.1e  E %.1e  grad %.1e  %s\n", name, E.H.passes.size(),
           E.H.lays.size(), E.H.fops.size(), max_state, max_e, max_g, ok ? "ok" : "FAIL");
}

int main(int argc, char** argv)
{
    const bool quick = argc > 1 && std::string(argv[1]) == "quick";
    std::mt19937_64 rng(7);
    for (int dt : {SV_C128, SV_C64})
        for (int apt : {16, 8})
            for (int wg : {0, 1}) {
                if (quick && apt == 8 && wg == 0) continue;
                char nm[128];
                snprintf(nm, sizeof nm, "hea 14q L4 %s apt%d grad%d", dt == SV_C128 ? "c128" : "c64", apt, wg);
                test({hea(14, 4)}, dt, 0, apt, wg, nm, rng);
                for (int tile : {4, 5, 6, 9}) {
                    if (quick && (tile == 5 || tile == 6)) continue;
                    snprintf(nm, sizeof nm, "random 10q tile%d %s apt%d grad%d", tile, dt == SV_C128 ? "c128" : "c64", apt, wg);
                    std::vector<Circ> cs;
                    for (int k = 0; k < 3; ++k) cs.push_back(random_circ(rng, 6 + 2 * k, 60, 5));
                    test(cs, dt, tile, apt, wg, nm, rng);
                }
                snprintf(nm, sizeof nm, "random 13q default tile %s apt%d grad%d", dt == SV_C128 ? "c128" : "c64", apt, wg);
                test({random_circ(rng, 13, 200, 12), random_circ(rng, 14, 150, 9)}, dt, 0, apt, wg, nm, rng);
                for (int tile : {4, 6}) {
                    snprintf(nm, sizeof nm, "cnot runs 11q tile%d %s apt%d grad%d", tile, dt == SV_C128 ? "c128" : "c64",
                             apt, wg);
                    test({cnot_runs(11), cnot_runs(9)}, dt, tile, apt, wg, nm, rng);
                }
                for (int tile : {5, 7, 0}) {
                    snprintf(nm, sizeof nm, "qft 11q + phases 12q tile%d %s apt%d grad%d", tile,
                             dt == SV_C128 ? "c128" : "c64", apt, wg);
                    test({qft(11), phase_heavy(rng, 12, 120, 6)}, dt, tile, apt, wg, nm, rng);
                }
            }
    printf("two-branch ops replayed: %ld with the selector on a lane bit, %ld on a register bit\n", pairc_lane,
           pairc_reg);
    printf("one-target ops with controls outside the tile replayed: %ld (tile x op)\n", gated_ops);
    printf("tile-selected ops replayed: %ld (tile x op)\n", tsel_ops);
    printf("subset phases replayed in per-target runs: %ld (tile x op)\n", run_members);
    printf("reverse pairs replayed: %ld (tile x op)\n", rfuse_ops);
    if (!rfuse_ops) {
        ++errors;
        printf("FAIL: the circuits do not exercise reverse pairs\n");
    }
    if (!run_members) {
        ++errors;
        printf("FAIL: the circuits do not exercise phase runs\n");
    }
    if (!tsel_ops) {
        ++errors;
        printf("FAIL: the circuits do not exercise tile-selected ops\n");
    }
    if (!gated_ops) {
        ++errors;
        printf("FAIL: the circuits do not exercise controls outside the tile\n");
    }
    if (!pairc_lane || !pairc_reg) {
        ++errors;
        printf("FAIL: the circuits do not exercise both selector placements of the two-branch op\n");
    }
    printf("%s (%d errors)\n", errors ? "FAILED" : "all ok", errors);
    return errors ? 1 : 0;
}

// sv_batch.hip -- host side of the fused pass engine: validation, the pass
// scheduler (gate fusion), table building, the persistent launch and its
// hipGraph capture.
//
// Pass scheduling.  Each op may move ahead of every earlier op it shares no
// qubit with (ops on disjoint qubits commute).  An op is ready when it is the
// next unscheduled op on each of its qubits.  A pass starts from the
// coalescing bits (the lowest bits, so a tile's loads cover whole 128-byte
// lines) and greedily takes ready ops in program order while the union of
// their qubits stays within tq qubits; it is then padded with the lowest
// unused qubits to exactly tq.  Every op of a pass acts inside one tile, so
// one HBM round trip of the state serves all of them.  A subset phase (Z, S,
// T, PHASE, any controls) is diagonal in every one of its qubits: its qubits
// outside the tile are fixed over a tile and only decide whether it acts
// there, so it joins a pass as soon as one of its qubits is in the tile (or
// its target can still be added), without growing the tile further.  The
// QFT's controlled phases then ride along with the Hadamard passes.
//
// Register tiling.  Inside a pass each thread holds 2^rb amplitudes of the
// tile.  The ops of the pass are grouped again (same commutation rule) into
// runs whose targets fit in rb register bits; each run gets a layout (which
// tile bits are register bits, and an order of the lane bits chosen for
// coalesced loads and conflict-free LDS exchange), and a layout change
// between runs is the only LDS step.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sv_core.h"
#include "sv_pass.h"

using namespace svk;

namespace {

struct BOp {
    int gate;
    int nc, nt;
    int q[SV_OP_MAX_QUBITS];
    int pidx;
    double value;
    std::vector<double> mat;
    uint64_t qmask() const
    {
        uint64_t m = 0;
        for (int j = 0; j < nc + nt; ++j) m |= 1ull << q[j];
        return m;
    }
};

int popc(uint64_t x) { return __builtin_popcountll(x); }

int targets_of(int gate) { return gate == SV_SWAP || gate == SV_U4 ? 2 : 1; }

// Subset phases: a phase on the amplitudes holding every qubit of the op.
bool subset_phase_gate(int gate) { return gate == SV_Z || gate == SV_S || gate == SV_T || gate == SV_PHASE; }

bool is_rotation(int gate) { return gate == SV_RX || gate == SV_RY || gate == SV_RZ || gate == SV_PHASE; }

sv_status validate(int n, const sv_op& s, int n_params, int index, BOp* out)
{
    const std::string at = "op " + std::to_string(index) + ": ";
    if (s.gate < SV_I || s.gate > SV_U4) return set_error(SV_ERR_ARG, at + "unknown gate");
    if (s.n_controls < 0 || s.n_controls > SV_MAX_CONTROLS) return set_error(SV_ERR_ARG, at + "bad control count");
    if (s.n_targets != targets_of(s.gate)) return set_error(SV_ERR_ARG, at + "wrong number of targets");
    uint64_t seen = 0;
    for (int j = 0; j < s.n_controls + s.n_targets; ++j) {
        const int q = s.qubits[j];
        if (q < 0 || q >= n) return set_error(SV_ERR_QUBIT, at + "qubit out of range");
        if (seen & (1ull << q)) return set_error(SV_ERR_QUBIT, at + "qubit repeated");
        seen |= 1ull << q;
    }
    if (s.param_index < -1 || s.param_index >= n_params) return set_error(SV_ERR_ARG, at + "parameter index out of range");
    if (s.param_index >= 0 && !is_rotation(s.gate)) return set_error(SV_ERR_ARG, at + "gate takes no parameter");
    if ((s.gate == SV_U2 || s.gate == SV_U4) && !s.matrix) return set_error(SV_ERR_ARG, at + "missing matrix");
    out->gate = s.gate;
    out->nc = s.n_controls;
    out->nt = s.n_targets;
    for (int j = 0; j < s.n_controls + s.n_targets; ++j) out->q[j] = s.qubits[j];
    out->pidx = s.param_index;
    out->value = s.value;
    if (s.gate == SV_U2) out->mat.assign(s.matrix, s.matrix + 8);
    if (s.gate == SV_U4) out->mat.assign(s.matrix, s.matrix + 32);
    return SV_OK;
}

// The qubits an op needs inside a pass's tile (P: the tile so far).  A subset
// phase joins on any one of its qubits (its target if none is in the tile).
// A one-target op needs its target only: a control outside the tile is
// constant over a tile, so it just selects the tiles the op acts on (the
// kernels test the tile index), as a control on a non-local qubit selects the
// processes that act in the paper's distributed scheme.  Two-target ops need
// all their qubits.
uint64_t tile_need(const BOp& o, uint64_t P, bool free_ctrl)
{
    if (subset_phase_gate(o.gate)) return (o.qmask() & P) ? 0ull : (1ull << o.q[o.nc]);
    if (o.nt == 1 && free_ctrl) return 1ull << o.q[o.nc];
    return o.qmask();
}

// Greedy commutation-aware grouping of ops into passes of at most tq qubits.
// With `reserve`, a qubit that joins the tile brings the other qubits of the
// next multi-qubit op on it (subset phases aside) when they still fit, so that
// op can follow in the same pass: a rotation and the CNOT ladder step onto its
// qubit land together (fewer passes for ladders, and the pair fuses).
void schedule_greedy(int n, int tq, int cb, const std::vector<BOp>& ops, bool reserve, bool free_ctrl,
                     std::vector<std::vector<int>>& pass_ops, std::vector<uint64_t>& pass_q)
{
    const int m = (int)ops.size();
    std::vector<std::vector<int>> qops(n);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < ops[i].nc + ops[i].nt; ++j) qops[ops[i].q[j]].push_back(i);
    std::vector<int> front(n, 0);
    std::vector<char> done(m, 0);
    int remaining = m, first = 0;
    const uint64_t cmask = cb > 0 ? ((1ull << cb) - 1ull) : 0ull;
    while (remaining > 0) {
        uint64_t P = cmask;
        int nparam = 0;
        std::vector<int> po;
        bool added = true;
        while (added) {
            added = false;
            while (first < m && done[first]) ++first;
            for (int i = first; i < m; ++i) {
                if (done[i]) continue;
                const BOp& o = ops[i];
                bool ready = true;
                for (int j = 0; j < o.nc + o.nt && ready; ++j) {
                    const int q = o.q[j];
                    ready = qops[q][front[q]] == i;
                }
                if (!ready) continue;
                const uint64_t np = P | tile_need(o, P, free_ctrl);
                if (popc(np) > tq) continue;
                if (o.pidx >= 0 && nparam >= kMaxPassSlots) continue;
                done[i] = 1;
                --remaining;
                po.push_back(i);
                const uint64_t grown = np & ~P;
                P = np;
                nparam += o.pidx >= 0;
                for (int j = 0; j < o.nc + o.nt; ++j) ++front[o.q[j]];
                added = true;
                if (reserve) {
                    for (uint64_t gq = grown; gq; gq &= gq - 1) {
                        const int q = __builtin_ctzll(gq);
                        for (size_t k = front[q]; k < qops[q].size(); ++k) {
                            const BOp& nx = ops[qops[q][k]];
                            if (subset_phase_gate(nx.gate)) continue;
                            if (nx.qmask() & ~(1ull << q)) {
                                const uint64_t r = P | tile_need(nx, P, free_ctrl);
                                if (popc(r) <= tq) P = r;
                                break;
                            }
                        }
                    }
                }
            }
        }
        for (int q = 0; q < n && popc(P) < tq; ++q) P |= 1ull << q;
        pass_ops.push_back(po);
        pass_q.push_back(P);
    }
}

// Four greedy forms, keeping the one with the fewest passes (the first of
// them on a tie): with or without reserving room for the next multi-qubit op
// of a joining qubit, and with controls of one-target ops inside the tile or
// left outside.  Reserving helps ladders (the 32-qubit HEA: 26 passes instead
// of 35); controls left outside help circuits whose controls range over the
// whole register (the 32-qubit universal circuit: 7 passes instead of 112)
// but leave the HEA's CNOTs unfused and take it to 32.
void schedule(int n, int tq, int cb, const std::vector<BOp>& ops, std::vector<std::vector<int>>& pass_ops,
              std::vector<uint64_t>& pass_q)
{
    bool have = false;
    for (int form = 0; form < 4; ++form) {
        std::vector<std::vector<int>> po;
        std::vector<uint64_t> pq;
        schedule_greedy(n, tq, cb, ops, (form & 1) != 0, (form & 2) != 0, po, pq);
        if (!have || po.size() < pass_ops.size()) {
            pass_ops.swap(po);
            pass_q.swap(pq);
            have = true;
        }
    }
}

// Tile bits an op needs in registers: the targets of pair ops and SWAP.
// Diagonal and subset-phase ops act element-wise in any layout; 4x4 ops are
// applied by a sweep over the LDS tile.
uint32_t op_need(const FOp& f)
{
    switch (f.kind) {
    case FK_PAIR:
    case FK_PAIRR:
    case FK_PAIRX:
    case FK_PAIRC:
    case FK_PAIRT:
    case FK_RFUSE: return 1u << f.a;
    case FK_SWAP: return (1u << f.a) | (1u << f.b);
    default: return 0u;
    }
}

uint32_t op_touch(const FOp& f)
{
    uint32_t m = f.cm | (1u << f.a);
    if (f.kind == FK_SWAP || f.kind == FK_QUAD || f.kind == FK_PAIRC) m |= 1u << f.b;
    return m;
}

// Fill a register set up to rb bits, highest free bits first, keeping the
// lowest `keep` bits (the coalescing run) as lane bits where possible.
uint32_t pad_regs(uint32_t S, int tq, int rb, int keep)
{
    for (int p = tq - 1; p >= keep && popc(S) < rb; --p) S |= 1u << p;
    for (int p = tq - 1; p >= 0 && popc(S) < rb; --p) S |= 1u << p;
    return S;
}

// Lane order: first up to kSwzBits lane bits with distinct residues mod
// kSwzBits, scanning upwards (so a coalescing run 0..cb-1 of lane bits comes
// first, in order), then the other lane bits ascending; register bits ascending.
FLayout make_layout(uint32_t S, int tq, int rb, const int32_t* q)
{
    FLayout L;
    memset(&L, 0, sizeof L);
    int lanes[16], nl = 0;
    bool used[16] = {}, res[kSwzBits] = {};
    for (int p = 0; p < tq && nl < kSwzBits; ++p) {
        if ((S >> p) & 1u) continue;
        if (res[p % kSwzBits]) continue;
        res[p % kSwzBits] = true;
        used[p] = true;
        lanes[nl++] = p;
    }
    for (int p = 0; p < tq; ++p)
        if (!((S >> p) & 1u) && !used[p]) lanes[nl++] = p;
    for (int i = 0; i < nl; ++i) L.pos[i] = (uint8_t)lanes[i];
    int r = 0;
    for (int p = 0; p < tq; ++p)
        if ((S >> p) & 1u) L.pos[(tq - rb) + r++] = (uint8_t)p;
    for (int i = 0; i < nl; ++i) {
        L.lane_l[i] = (uint16_t)(1u << L.pos[i]);
        L.lane_g[i] = 1ull << q[L.pos[i]];
    }
    for (int k = 0; k < rb; ++k) {
        L.reg_l[k] = (uint16_t)(1u << L.pos[nl + k]);
        L.reg_g[k] = 1ull << q[L.pos[nl + k]];
    }
    return L;
}

int reg_index(uint32_t S, int p) { return popc(S & ((1u << p) - 1u)); }

// Reorder one pass's ops into register runs and insert the layout changes.
void plan_layouts(std::vector<FOp>& pass_ops, int tq, int rb, int cb, const int32_t* q, std::vector<FLayout>& lays,
                  int& lay_begin, int& lay_end)
{
    const int keep = std::max(0, std::min(cb, tq - rb));
    const uint32_t lowmask = (1u << keep) - 1u;
    std::vector<std::pair<uint32_t, std::vector<int>>> runs;
    std::vector<int> remaining(pass_ops.size());
    for (size_t i = 0; i < pass_ops.size(); ++i) remaining[i] = (int)i;
    while (!remaining.empty()) {
        uint32_t S = 0, blocked = 0;
        std::vector<int> taken, rest;
        for (int i : remaining) {
            const FOp& f = pass_ops[i];
            const uint32_t m = op_touch(f);
            if (m & blocked) {
                blocked |= m;
                rest.push_back(i);
                continue;
            }
            const uint32_t nd = op_need(f);
            if (popc(S | nd) <= rb) {
                S |= nd;
                taken.push_back(i);
            } else {
                blocked |= m;
                rest.push_back(i);
            }
        }
        runs.push_back({pad_regs(S, tq, rb, keep), taken});
        remaining.swap(rest);
    }
    const uint32_t C = pad_regs(0, tq, rb, keep);
    std::vector<std::pair<uint32_t, int>> seen;  // register set -> layout index (this pass)
    auto layout_of = [&](uint32_t S) {
        for (auto& e : seen)
            if (e.first == S) return e.second;
        lays.push_back(make_layout(S, tq, rb, q));
        seen.push_back({S, (int)lays.size() - 1});
        return (int)lays.size() - 1;
    };
    std::vector<FOp> out;
    auto marker = [&](int to, int from) {
        FOp m;
        memset(&m, 0, sizeof m);
        m.kind = FK_LAYOUT;
        m.a = to;
        m.b = from;
        m.slot = -1;
        out.push_back(m);
    };
    int cur;
    if (runs.empty() || (runs[0].first & lowmask)) cur = layout_of(C);
    else cur = layout_of(runs[0].first);
    lay_begin = cur;
    for (auto& r : runs) {
        const int li = layout_of(r.first);
        if (li != cur) {
            marker(li, cur);
            cur = li;
        }
        for (int i : r.second) {
            FOp f = pass_ops[i];
            const uint32_t S = r.first;
            f.ka = (int8_t)(((S >> f.a) & 1u) ? reg_index(S, f.a) : -1);
            const bool two = f.kind == FK_SWAP || f.kind == FK_QUAD || f.kind == FK_PAIRC;
            f.kb = (int8_t)(two && ((S >> f.b) & 1u) ? reg_index(S, f.b) : -1);
            uint32_t cmk = 0;
            for (int q = 0; q < 32; ++q)
                if (((f.cm & S) >> q) & 1u) cmk |= 1u << reg_index(S, q);
            f.cmk = (uint8_t)cmk;
            f.cml = f.cm & ~S;
            out.push_back(f);
        }
    }
    if (!runs.empty() && (runs.back().first & lowmask)) {
        const int li = layout_of(C);
        if (li != cur) {
            marker(li, cur);
            cur = li;
        }
    }
    lay_end = cur;
    pass_ops.swap(out);
}

bool diag_gate(int g) { return g == SV_RZ || g == SV_PHASE || g == SV_Z || g == SV_S || g == SV_T; }
bool real_gate(int g) { return g == SV_RY || g == SV_H || g == SV_X || g == SV_Z; }
bool one_target_kind(int k) { return k == FK_PAIR || k == FK_PAIRR || k == FK_PAIRX || k == FK_DIAG || k == FK_PHASE; }

// Factor entry of a one-target gate: rotations are evaluated from their
// parameter on the device, fixed gates carry their full 2x2.
FCoefSpec factor_of(const BOp& o, int param_base)
{
    FCoefSpec f;
    memset(&f, 0, sizeof f);
    f.gate = o.gate;
    f.pidx = o.pidx >= 0 ? param_base + o.pidx : -1;
    f.value = o.value;
    const double r = M_SQRT1_2;
    double m[8] = {1, 0, 0, 0, 0, 0, 1, 0};
    switch (o.gate) {
    case SV_X: { const double x[8] = {0, 0, 1, 0, 1, 0, 0, 0}; memcpy(m, x, sizeof m); break; }
    case SV_Y: { const double x[8] = {0, 0, 0, -1, 0, 1, 0, 0}; memcpy(m, x, sizeof m); break; }
    case SV_H: { const double x[8] = {r, 0, r, 0, r, 0, -r, 0}; memcpy(m, x, sizeof m); break; }
    case SV_U2: memcpy(m, o.mat.data(), sizeof m); break;
    case SV_Z: m[6] = -1; break;
    case SV_S: m[6] = 0; m[7] = 1; break;
    case SV_T: m[6] = cos(M_PI / 4); m[7] = sin(M_PI / 4); break;
    default: break;  // rotations: evaluated on the device
    }
    memcpy(f.fixed, m, sizeof m);
    return f;
}

// Forward-list gate fusion: a one-target op joins the previous op on the same
// target when it may move back to that op (no op in between touches any of
// its qubits: ops on disjoint qubits commute) and
//   * it has the group's controls (a group without a selector), or
//   * it has one control s and the group has none: the group becomes a
//     two-branch group with selector s, and the op enters only the branch
//     where s is 1 (a rotation followed by a CNOT from s becomes one op whose
//     2x2 is U where s is 0 and X U where s is 1), or
//   * the group has a selector s and the op is uncontrolled (both branches)
//     or controlled by s alone (the second branch), or
//   * the group's ops all have the one control s and the op is uncontrolled:
//     the group becomes two-branch, its ops in the second branch and the op
//     in both (a CNOT followed by a rotation of its target), or
//   * neither the group nor the op has a control inside the tile, and the
//     union of their controls outside it stays within kMaxTileSelBits: the
//     group becomes tile-selected (FK_PAIRT), one product per combination of
//     those bits, each gate entering the products whose combination holds
//     all of its controls (a run of CNOTs from far qubits interleaved with
//     rotations of their common target).
// A group of more than one op becomes one op whose coefficients are the
// product of its gates, per branch (evaluated on the device from the
// parameters).  Reverse passes keep the ops unfused: each parameterised op
// needs its own gradient partial.
std::vector<FOp> fuse_forward(const std::vector<FOp>& ops, const std::vector<int>& src, const std::vector<BOp>& bops,
                              int param_base, std::vector<FCoefSpec>& cspec, std::vector<FCoefSpec>& cfac,
                              int& coef_total)
{
    struct Grp {
        FOp op;
        uint32_t ctrl;
        bool fusable;
        int sel;                   // selector bit of a two-branch group, -1 if none
        std::vector<int> members;  // indices into bops
        std::vector<int> branch;   // per member: 3 both branches, 2 the selector-1 branch
        std::vector<uint32_t> out; // per member: its controls outside the tile (packed)
        uint32_t tmask;            // union of the members' controls outside the tile
    };
    std::vector<Grp> g;
    int last[32];
    for (int& x : last) x = -1;
    for (size_t i = 0; i < ops.size(); ++i) {
        const FOp& f = ops[i];
        // a subset phase with qubits outside the tile stays on its own (it may be
        // chained); a one-target gate with controls outside the tile may join a
        // group whose controls also lie outside the tile
        const uint32_t ctrl = f.kind == FK_PHASE ? (f.cm & ~(1u << f.a)) : f.cm;
        const bool fus = one_target_kind(f.kind) && (f.b == 0 || (f.kind != FK_PHASE && ctrl == 0));
        uint32_t touch = f.cm | (1u << f.a);
        if (f.kind == FK_SWAP || f.kind == FK_QUAD) touch |= 1u << f.b;
        if (fus) {
            const int c = last[f.a];
            if (c >= 0 && g[c].fusable && g[c].op.a == f.a) {
                Grp& G = g[c];
                bool later = false;  // a later group touched one of the op's qubits
                for (int q = 0; q < 32; ++q)
                    if ((touch >> q) & 1u) later = later || last[q] != c;
                int tag = 0;
                if (f.b != 0 || G.tmask != 0) {
                    // tile-selected: no control inside the tile on either side
                    if (G.sel < 0 && G.ctrl == 0 && ctrl == 0 && popc(G.tmask | (uint32_t)f.b) <= kMaxTileSelBits) {
                        G.tmask |= (uint32_t)f.b;
                        G.members.push_back(src[i]);
                        G.branch.push_back(3);
                        G.out.push_back((uint32_t)f.b);
                        continue;
                    }
                } else if (G.sel < 0 && G.ctrl == ctrl && !later) {
                    tag = 3;
                } else if (G.sel >= 0 && ctrl == 0) {
                    tag = 3;  // touches only the target, whose latest group is G
                } else if (G.sel >= 0 && ctrl == (1u << G.sel) && !later) {
                    tag = 2;
                } else if (G.sel < 0 && G.ctrl == 0 && popc(ctrl) == 1 && last[__builtin_ctz(ctrl)] <= c) {
                    G.sel = __builtin_ctz(ctrl);  // no later group touched it: the op moves back to G
                    last[G.sel] = c;
                    tag = 2;
                } else if (G.sel < 0 && popc(G.ctrl) == 1 && ctrl == 0) {
                    // a group controlled by one qubit s, then an uncontrolled op:
                    // the group's ops become the s = 1 branch
                    G.sel = __builtin_ctz(G.ctrl);
                    G.ctrl = 0;
                    for (int& b : G.branch) b = 2;
                    tag = 3;
                }
                if (tag) {
                    G.members.push_back(src[i]);
                    G.branch.push_back(tag);
                    G.out.push_back(0u);
                    continue;
                }
            }
        }
        const uint32_t out_bits = fus ? (uint32_t)f.b : 0u;
        g.push_back({f, ctrl, fus, -1, {src[i]}, {3}, {out_bits}, out_bits});
        for (int q = 0; q < 32; ++q)
            if ((touch >> q) & 1u) last[q] = (int)g.size() - 1;
    }
    std::vector<FOp> out;
    for (Grp& gr : g) {
        if (gr.members.size() == 1) {
            out.push_back(gr.op);
            continue;
        }
        bool all_diag = true, all_real = true;
        for (int m : gr.members) {
            all_diag = all_diag && diag_gate(bops[m].gate);
            all_real = all_real && real_gate(bops[m].gate);
        }
        const bool two = gr.sel >= 0, tsel = gr.tmask != 0;
        FOp f = gr.op;
        f.kind = tsel ? FK_PAIRT : two ? FK_PAIRC : (all_diag ? FK_DIAG : (all_real ? FK_PAIRR : FK_PAIR));
        f.cm = gr.ctrl;
        if (two) f.b = gr.sel;
        if (tsel) f.b = (int32_t)gr.tmask;
        f.slot = -1;
        f.coef = coef_total;
        FCoefSpec cs;
        memset(&cs, 0, sizeof cs);
        cs.gate = SV_I;
        cs.pidx = -1;
        cs.coef = coef_total;
        cs.nfactor = (int)gr.members.size();
        cs.factor_begin = (int)cfac.size();
        cs.out_diag = tsel ? 3 : two ? 2 : (all_diag ? 1 : 0);
        if (tsel) cs.branch = (int32_t)gr.tmask;
        for (size_t k = 0; k < gr.members.size(); ++k) {
            FCoefSpec fa = factor_of(bops[gr.members[k]], param_base);
            fa.branch = tsel ? (int32_t)gr.out[k] : gr.branch[k];
            cfac.push_back(fa);
        }
        cspec.push_back(cs);
        coef_total += tsel ? 8 << popc(gr.tmask) : two ? 16 : (all_diag ? 4 : 8);
        out.push_back(f);
    }
    return out;
}

}  // namespace

struct sv_batch_s {
    int dtype;
    hipStream_t stream;
    int n_circ;
    int with_grad;
    int use_graph;
    int threads, rthreads;
    int reg_bits, rreg_bits;
    size_t lds_fwd, lds_rev;  // dynamic LDS of forward and reverse workgroups
    std::vector<int64_t> level_first;  // per level: forward, observable, reverse item ranges (4 bounds)
    std::vector<uint8_t> level_gated;  // per level: 1 if a forward pass of the level has FPass.gated set
    int64_t n_items;
    int n_segs;
    int n_slots;
    int n_params;
    int n_passes;
    int max_passes;
    int n_fops;  // gate ops scheduled
    int n_layout_changes;
    int n_levels;
    size_t state_bytes;
    double pass_bytes;  // HBM bytes of all passes of one run (algorithmic)
    std::vector<size_t> psi_off;
    std::vector<int> nq;
    PassTables tb;
    // device allocations
    void* d_psi;
    void* d_lam;
    FCirc* d_circ;
    FPass* d_pass;
    FOp* d_ops;
    FLayout* d_lays;
    FSeg* d_segs;
    FCoefSpec* d_cspec;
    FCoefSpec* d_cfac;
    int n_cspec;
    double* d_coef;
    float* d_coef_f;
    double* d_epart;
    double* d_gpart;
    int64_t* d_e_off;
    int* d_e_cnt;
    int64_t* d_g_off;
    int* d_g_cnt;
    double* d_slot_scale;
    double* d_slot_val;
    int* d_csr_ptr;
    int* d_csr_col;
    double* d_params;
    double* d_expvals;
    double* d_grads;
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool graph_ready;
    // the caller's stream (sv_batch_set_stream; default the null stream): a
    // run waits for the work queued there before it, and work queued there
    // after the run waits for the run's outputs
    hipStream_t caller;
    hipEvent_t ev_in, ev_out;
};

namespace {

template <typename X>
hipError_t dev_upload(X** dst, const std::vector<X>& src)
{
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(X);
    hipError_t e = hipMalloc((void**)dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(X), hipMemcpyHostToDevice);
    return e;
}

void batch_release(sv_batch b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    void* ptrs[] = {b->d_psi, b->d_lam, b->d_circ, b->d_pass, b->d_ops, b->d_lays, b->d_segs, b->d_cspec, b->d_cfac, b->d_coef, b->d_coef_f, b->d_epart, b->d_gpart, b->d_e_off, b->d_e_cnt, b->d_g_off, b->d_g_cnt,
                    b->d_slot_scale, b->d_slot_val, b->d_csr_ptr, b->d_csr_col, b->d_params, b->d_expvals,
                    b->d_grads};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

hipError_t enqueue_run(sv_batch b)
{
    hipStream_t s = b->stream;
    hipError_t e = launch_pass_coef(b->d_cspec, b->n_cspec, b->d_cfac, b->d_params, b->d_coef,
                                    b->dtype == SV_C64 ? b->d_coef_f : nullptr, s);
    const std::vector<int64_t>& lf = b->level_first;
    for (size_t l = 0; l + 3 < lf.size() && e == hipSuccess; l += 3) {
        e = launch_pass_items(b->tb, b->dtype, PM_FWD, lf[l], lf[l + 1], b->threads, b->lds_fwd, s,
                              b->level_gated[l / 3] != 0);
        if (e == hipSuccess) e = launch_pass_items(b->tb, b->dtype, PM_OBS, lf[l + 1], lf[l + 2], b->threads, 0, s);
        if (e == hipSuccess)
            e = launch_pass_items(b->tb, b->dtype, PM_REV, lf[l + 2], lf[l + 3], b->rthreads, b->lds_rev, s);
    }
    if (e == hipSuccess) e = launch_pass_segsum(b->d_epart, b->d_e_off, b->d_e_cnt, nullptr, b->d_expvals, b->n_circ, s);
    if (e == hipSuccess && b->with_grad) {
        e = launch_pass_segsum(b->d_gpart, b->d_g_off, b->d_g_cnt, b->d_slot_scale, b->d_slot_val, b->n_slots, s);
        if (e == hipSuccess) e = launch_pass_grad_csr(b->d_slot_val, b->d_csr_ptr, b->d_csr_col, b->n_params, b->d_grads, s);
    }
    return e;
}

// Reverse-list fusion: a one-target gate B joins the earlier gate A on the
// same target with the same in-tile controls (and none outside the tile)
// when no op in between touches their qubits, so B may move back to A (ops
// on disjoint qubits commute, and so do their gradient terms).  The pair
// becomes one FK_RFUSE op: one un-apply of B A on phi and lambda, B's
// gradient partial with its own generator and A's with B G_A B^dagger, both
// taken before the un-apply.  Subset phases, gated and two-target ops stay
// as they are.
std::vector<FOp> fuse_reverse(const std::vector<FOp>& ops, const std::vector<int>& src, const std::vector<BOp>& bops,
                              int param_base, std::vector<FCoefSpec>& cspec, std::vector<FCoefSpec>& cfac,
                              int& coef_total)
{
    struct Grp {
        int first, second;
        bool fusable;
    };
    std::vector<Grp> g;
    int last[32];
    for (int& x : last) x = -1;
    auto eligible = [](const FOp& f) {
        return (f.kind == FK_PAIR || f.kind == FK_PAIRR || f.kind == FK_PAIRX || f.kind == FK_DIAG) && f.b == 0;
    };
    for (size_t i = 0; i < ops.size(); ++i) {
        const FOp& f = ops[i];
        uint32_t touch = f.cm | (1u << f.a);
        if (f.kind == FK_SWAP || f.kind == FK_QUAD || f.kind == FK_PAIRC) touch |= 1u << f.b;
        if (eligible(f)) {
            const int c = last[f.a];
            if (c >= 0 && g[c].fusable && g[c].second < 0 && ops[g[c].first].a == f.a && ops[g[c].first].cm == f.cm) {
                bool later = false;
                for (int q = 0; q < 32; ++q)
                    if ((touch >> q) & 1u) later = later || last[q] != c;
                if (!later) {
                    g[c].second = (int)i;
                    continue;
                }
            }
        }
        g.push_back({(int)i, -1, eligible(f)});
        for (int q = 0; q < 32; ++q)
            if ((touch >> q) & 1u) last[q] = (int)g.size() - 1;
    }
    std::vector<FOp> out;
    for (const Grp& gr : g) {
        if (gr.second < 0) {
            out.push_back(ops[gr.first]);
            continue;
        }
        const FOp& A = ops[gr.first];
        const FOp& B = ops[gr.second];
        FOp f = B;
        f.kind = FK_RFUSE;
        f.b = A.slot;
        f.coef = coef_total;
        FCoefSpec cs;
        memset(&cs, 0, sizeof cs);
        cs.gate = SV_I;
        cs.pidx = -1;
        cs.coef = coef_total;
        cs.nfactor = 2;
        cs.factor_begin = (int)cfac.size();
        cs.out_diag = 4;
        cs.branch = A.slot >= 0 ? 1 + A.gen : 0;
        cfac.push_back(factor_of(bops[src[gr.first]], param_base));
        cfac.push_back(factor_of(bops[src[gr.second]], param_base));
        cspec.push_back(cs);
        coef_total += 16;
        out.push_back(f);
    }
    return out;
}

// Consecutive subset phases commute.  Within each maximal run of them in a
// planned forward list (no layout change inside, so one local mask means one
// register / lane split) the host groups them:
//   * a phase whose in-tile mask is one bit t, or t and one lane bit c, joins
//     the group of run target t (for a mask of one register bit and one lane
//     bit, t is the register bit): the kernel multiplies the group's phases
//     into one factor per lane (a member with c counts on the lanes holding
//     c) and applies it once to the amplitudes holding t.  Members carry
//     a = t (ka to match) and kb = 2, the last one kb = 3;
//   * other phases are ordered by local mask and each is chained to the next
//     of the same mask (kb = 1): the kernel multiplies a chain's phases (those
//     whose out-of-tile bits the tile holds) into one and applies it once.
// Changing a phase's named target changes nothing: a subset phase is
// symmetric in the qubits of its mask.
void mark_phase_chains(std::vector<FOp>& ops)
{
    auto run_target = [](const FOp& f) -> int {
        const uint32_t reg = f.cm & ~f.cml;  // in-tile bits on registers (cml: those on lanes)
        const int n = popc(f.cm);
        if (n == 1) return f.a;
        if (n != 2 || popc(reg) == 2) return -1;
        return popc(reg) == 1 ? __builtin_ctz(reg) : f.a;
    };
    size_t i = 0;
    while (i < ops.size()) {
        if (ops[i].kind != FK_PHASE) {
            ++i;
            continue;
        }
        size_t j = i;
        while (j < ops.size() && ops[j].kind == FK_PHASE) ++j;
        // run groups first, by target; then the others by mask
        auto key = [&](const FOp& f) {
            const int t = run_target(f);
            return t >= 0 ? (int64_t)t : (int64_t)64 + (int64_t)f.cm;
        };
        std::stable_sort(ops.begin() + i, ops.begin() + j, [&](const FOp& x, const FOp& y) { return key(x) < key(y); });
        for (size_t k = i; k < j;) {
            size_t e = k;
            while (e < j && key(ops[e]) == key(ops[k])) ++e;
            const int t = run_target(ops[k]);
            if (t >= 0 && e - k >= 2) {
                for (size_t m = k; m < e; ++m) {
                    FOp& f = ops[m];
                    const bool treg = ((f.cm & ~f.cml) >> t) & 1u;
                    f.a = t;
                    f.ka = (int8_t)(treg ? __builtin_ctz(f.cmk) : -1);
                    f.kb = m + 1 < e ? 2 : 3;
                }
            } else {
                for (size_t m = k; m < e; ++m) ops[m].kb = (t < 0 && m + 1 < e) ? 1 : 0;
            }
            k = e;
        }
        i = j;
    }
}

}  // namespace

static sv_status hip_fail(hipError_t e, const char* what)
{
    return set_error(SV_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Everything a batch needs, built on the host (no device work).
struct HostTables {
    int tq_max, threads, rthreads, reg_bits, rreg_bits, lds_small, with_grad, cbits_default, n_params, coef_total,
        tq_used, hi_entries, e_total, n_levels, n_gate_ops, n_layout_changes;
    int64_t g_total, n_items;
    size_t state_total;
    double pass_bytes;
    std::vector<FCirc> circs;
    std::vector<FPass> passes;
    std::vector<FOp> fops;
    std::vector<FLayout> lays;
    std::vector<FCoefSpec> cspec, cfac;
    std::vector<double> slot_scale;
    std::vector<int> slot_param;
    std::vector<int64_t> g_off, e_off, level_first;
    std::vector<uint8_t> level_gated;
    std::vector<int> g_cnt, e_cnt, csr_ptr, csr_col;
    std::vector<FSeg> segs;
    std::vector<size_t> psi_off;
};

// Engine tile shape per dtype (index 0 complex64, 1 complex128) and stage mix
// (index 0 forward only, 1 with the adjoint sweep) used where sv_batch_opts
// leaves a field 0; 0 here means the built-in default.
static int g_engine_tq[2][2] = {{0, 0}, {0, 0}};
static int g_engine_apt[2][2] = {{0, 0}, {0, 0}};

// Largest tile whose forward workgroups (and reverse ones, with the adjoint)
// stay within kMaxPassThreads.
static int engine_tq_fit(int reg_bits, int rreg_bits, int with_grad)
{
    int lg_threads = 0;
    while ((2 << lg_threads) <= kMaxPassThreads) ++lg_threads;
    return (with_grad ? std::min(reg_bits, rreg_bits) : reg_bits) + lg_threads;
}

static sv_status compile_batch(const sv_batch_circuit* circuits, int n_circuits, int dtype, const sv_batch_opts* opts,
                               HostTables& H)
{
    if (!circuits || n_circuits < 1) return set_error(SV_ERR_ARG, "bad batch arguments");
    if (dtype != SV_C64 && dtype != SV_C128) return set_error(SV_ERR_ARG, "bad dtype");
    const int d = dtype == SV_C128 ? 1 : 0;
    const int with_grad = opts ? (opts->with_grad != 0) : 1;
    const int apt = opts && opts->amps_per_thread > 0 ? opts->amps_per_thread
                    : g_engine_apt[d][with_grad] > 0   ? g_engine_apt[d][with_grad]
                                                       : (1 << kMaxRegBits);
    int reg_bits = 0;
    for (int r = kMinRegBits; r <= kMaxRegBits; ++r)
        if (apt == (1 << r)) reg_bits = r;
    if (!reg_bits) return set_error(SV_ERR_ARG, "amps_per_thread must be 8 or 16");
    // reverse passes hold phi and lambda: complex128 keeps 8 amplitudes of each per thread
    const int rreg_bits = dtype == SV_C128 ? std::min(reg_bits, 3) : reg_bits;
    // default tile: the tuned one, else 64 KiB (2^12 complex128 / 2^13 complex64
    // amplitudes); either within kMaxPassThreads threads of the narrower register width
    const int tq_base = g_engine_tq[d][with_grad] > 0 ? g_engine_tq[d][with_grad] : (dtype == SV_C128 ? 12 : 13);
    const int tq_default = std::min(tq_base, engine_tq_fit(reg_bits, rreg_bits, with_grad));
    int tq_max = opts && opts->tile_qubits > 0 ? opts->tile_qubits : tq_default;
    if (tq_max < 2 || tq_max > kMaxTileQubits) return set_error(SV_ERR_ARG, "tile_qubits must be in [2, 13]");
    const int cbits_default = dtype == SV_C128 ? 3 : 4;  // 128-byte runs

    // ---- validate and schedule ----------------------------------------------------
    std::vector<FCirc> circs(n_circuits);
    std::vector<FPass> passes;
    std::vector<FOp> fops;
    std::vector<FLayout> lays;
    std::vector<FCoefSpec> cspec, cfac;
    std::vector<double> slot_scale;
    std::vector<int> slot_param;  // global parameter of each global slot
    std::vector<int64_t> g_off;
    std::vector<int> g_cnt;
    std::vector<int64_t> e_off;
    std::vector<int> e_cnt;
    std::vector<size_t> psi_off(n_circuits);
    int n_params = 0, coef_total = 0, tq_used = 2, hi_entries = 1, lds_small = 0;
    int64_t g_total = 0;
    int e_total = 0;
    size_t state_total = 0;
    double pass_bytes = 0;
    const size_t eb = dtype == SV_C128 ? 16 : 8;
    for (int c = 0; c < n_circuits; ++c) {
        const sv_batch_circuit& bc = circuits[c];
        if (bc.n_qubits < 1 || bc.n_qubits > SV_MAX_QUBITS || bc.n_ops < 0 || (bc.n_ops > 0 && !bc.ops) ||
            bc.n_params < 0 || (bc.obs_kind != 1 && bc.obs_kind != 2))
            return set_error(SV_ERR_ARG, "circuit " + std::to_string(c) + ": bad description");
        const int n = bc.n_qubits;
        std::vector<BOp> ops;
        int max_q = 1;
        for (int i = 0; i < bc.n_ops; ++i) {
            BOp o;
            sv_status rc = validate(n, bc.ops[i], bc.n_params, i, &o);
            if (rc) return set_error(rc, "circuit " + std::to_string(c) + ": " + sv_last_error());
            if (o.gate == SV_I) continue;
            max_q = std::max(max_q, o.nc + o.nt);
            ops.push_back(o);
        }
        const int tq = std::min(n, tq_max);
        if (max_q > tq) return set_error(SV_ERR_UNSUPPORTED, "circuit " + std::to_string(c) + ": an op has more qubits than a tile");
        const int cb = std::max(0, std::min(cbits_default, tq - max_q));
        std::vector<std::vector<int>> pops;
        std::vector<uint64_t> pq;
        schedule(n, tq, cb, ops, pops, pq);
        if (pops.empty()) {  // no ops: one empty pass still builds |0..0>
            pops.push_back({});
            uint64_t P = 0;
            for (int q = 0; q < tq; ++q) P |= 1ull << q;
            pq.push_back(P);
        }
        FCirc& fc = circs[c];
        memset(&fc, 0, sizeof fc);
        fc.n = n;
        fc.tq = tq;
        fc.cb = cb;
        fc.reg = tq >= reg_bits ? 1 : 0;
        fc.rreg = tq >= rreg_bits ? 1 : 0;
        if (!fc.reg || (with_grad && !fc.rreg)) {
            lds_small = 1;
            hi_entries = std::max(hi_entries, 1 << (tq - cb));
        }
        fc.n_tiles = 1 << (n - tq);
        fc.n_pass = (int)pops.size();
        fc.pass_begin = (int)passes.size();
        fc.obs_kind = bc.obs_kind;
        fc.e_part_begin = e_total;
        fc.g_part_begin = g_total;
        e_off.push_back(e_total);
        e_cnt.push_back(fc.n_tiles);
        e_total += fc.n_tiles;
        tq_used = std::max(tq_used, tq);
        int slot = 0;
        std::vector<int> slot_of(ops.size(), -1);
        for (size_t i = 0; i < ops.size(); ++i)
            if (ops[i].pidx >= 0) slot_of[i] = slot++;
        for (size_t p = 0; p < pops.size(); ++p) {
            FPass fp;
            memset(&fp, 0, sizeof fp);
            int local[64];
            int k = 0;
            for (int q = 0; q < 64; ++q) local[q] = -1;
            for (int q = 0; q < n; ++q)
                if (pq[p] & (1ull << q)) {
                    local[q] = k;
                    fp.q[k++] = q;
                }
            fp.free_mask = (n >= 64 ? ~0ull : ((1ull << n) - 1ull)) & ~pq[p];
            std::vector<FOp> pass_ops;
            std::vector<int> pass_src;
            for (int i : pops[p]) {
                const BOp& o = ops[i];
                FOp f;
                memset(&f, 0, sizeof f);
                f.slot = slot_of[i];
                f.gen = (int8_t)(o.gate == SV_RX ? GEN_X : (o.gate == SV_RY ? GEN_Y : (o.gate == SV_RZ ? GEN_Z : GEN_P1)));
                // controls (and a subset phase's target) inside the tile -> cm,
                // those outside it -> gm (a one-target op's tile gate)
                const bool sp = subset_phase_gate(o.gate);
                uint32_t cm = 0;
                uint64_t gm = 0;
                for (int j = 0; j < o.nc + (sp ? 1 : 0); ++j) {
                    const int q = o.q[j];
                    if (local[q] >= 0) cm |= 1u << local[q];
                    else gm |= 1ull << q;
                }
                const int tl0 = local[o.q[o.nc]];
                if ((!sp && (tl0 < 0 || (o.nt > 1 && (gm || local[o.q[o.nc + 1]] < 0)))) || (sp && !cm))
                    return set_error(SV_ERR_UNSUPPORTED, "internal: an op of a pass lies outside its tile");
                f.cm = cm;
                // a subset phase is symmetric in its qubits: any one inside the tile serves as its target
                f.a = tl0 >= 0 ? tl0 : __builtin_ctz(cm);
                f.b = o.nt > 1 ? local[o.q[o.nc + 1]] : 0;
                if (o.nt == 1) {  // b: the op's qubits outside the tile, packed as in a tile index (0: none)
                    uint32_t packed = 0;
                    for (int q = 0; q < n; ++q)
                        if ((gm >> q) & 1ull) packed |= 1u << popc(fp.free_mask & ((1ull << q) - 1ull));
                    f.b = (int32_t)packed;
                }
                FCoefSpec cs;
                memset(&cs, 0, sizeof cs);
                cs.gate = o.gate;
                cs.pidx = o.pidx >= 0 ? n_params + o.pidx : -1;
                cs.value = o.value;
                cs.coef = coef_total;
                f.coef = coef_total;
                const double r = M_SQRT1_2;
                switch (o.gate) {
                case SV_X: { f.kind = FK_PAIRX; double m[8] = {0, 0, 1, 0, 1, 0, 0, 0}; memcpy(cs.fixed, m, sizeof m); cs.nfixed = 8; coef_total += 8; break; }
                case SV_Y: { f.kind = FK_PAIR; double m[8] = {0, 0, 0, -1, 0, 1, 0, 0}; memcpy(cs.fixed, m, sizeof m); cs.nfixed = 8; coef_total += 8; break; }
                case SV_H: { f.kind = FK_PAIRR; double m[8] = {r, 0, r, 0, r, 0, -r, 0}; memcpy(cs.fixed, m, sizeof m); cs.nfixed = 8; coef_total += 8; break; }
                case SV_U2: { f.kind = FK_PAIR; memcpy(cs.fixed, o.mat.data(), 8 * sizeof(double)); cs.nfixed = 8; coef_total += 8; break; }
                case SV_RX: f.kind = FK_PAIR; coef_total += 8; break;
                case SV_RY: f.kind = FK_PAIRR; coef_total += 8; break;
                case SV_RZ: f.kind = FK_DIAG; coef_total += 4; break;
                case SV_Z: { f.kind = FK_PHASE; cs.fixed[0] = -1; cs.nfixed = 2; coef_total += 2; break; }
                case SV_S: { f.kind = FK_PHASE; cs.fixed[1] = 1; cs.nfixed = 2; coef_total += 2; break; }
                case SV_T: { f.kind = FK_PHASE; cs.fixed[0] = cos(M_PI / 4); cs.fixed[1] = sin(M_PI / 4); cs.nfixed = 2; coef_total += 2; break; }
                case SV_PHASE: f.kind = FK_PHASE; coef_total += 2; break;
                case SV_SWAP: f.kind = FK_SWAP; break;
                default: { f.kind = FK_QUAD; memcpy(cs.fixed, o.mat.data(), 32 * sizeof(double)); cs.nfixed = 32; coef_total += 32; break; }
                }
                if (o.gate != SV_SWAP) cspec.push_back(cs);
                pass_ops.push_back(f);
                pass_src.push_back(i);
            }
            std::vector<FOp> fwd_ops = fuse_forward(pass_ops, pass_src, ops, n_params, cspec, cfac, coef_total);
            const bool fused = fwd_ops.size() != pass_ops.size();
            if (fc.reg) {
                plan_layouts(fwd_ops, tq, reg_bits, cb, fp.q, lays, fp.lay_begin, fp.lay_end);
                mark_phase_chains(fwd_ops);
            }
            fp.op_begin = (int)fops.size();
            fops.insert(fops.end(), fwd_ops.begin(), fwd_ops.end());
            fp.op_end = (int)fops.size();
            fp.gated = 0;
            for (const FOp& f : fwd_ops)
                if ((f.b != 0 && (f.kind == FK_PAIR || f.kind == FK_PAIRR || f.kind == FK_PAIRX || f.kind == FK_DIAG)) ||
                    f.kind == FK_PAIRT)
                    fp.gated = 1;
            fp.rop_begin = fp.op_begin;
            fp.rop_end = fp.op_end;
            fp.rlay_begin = fp.lay_begin;
            fp.rlay_end = fp.lay_end;
            std::vector<FOp> rev_ops;
            if (with_grad && fc.rreg) rev_ops = fuse_reverse(pass_ops, pass_src, ops, n_params, cspec, cfac, coef_total);
            const bool rfused = with_grad && fc.rreg && rev_ops.size() != pass_ops.size();
            if (with_grad && (fused || rfused || fc.reg != fc.rreg || (fc.rreg && rreg_bits != reg_bits))) {
                if (!rfused) rev_ops = pass_ops;
                if (fc.rreg) plan_layouts(rev_ops, tq, rreg_bits, cb, fp.q, lays, fp.rlay_begin, fp.rlay_end);
                fp.rop_begin = (int)fops.size();
                fops.insert(fops.end(), rev_ops.begin(), rev_ops.end());
                fp.rop_end = (int)fops.size();
            }
            passes.push_back(fp);
        }
        for (size_t i = 0; i < ops.size(); ++i)
            if (ops[i].pidx >= 0) {
                slot_scale.push_back(ops[i].gate == SV_PHASE ? -2.0 : 1.0);
                slot_param.push_back(n_params + ops[i].pidx);
                g_off.push_back(g_total + (int64_t)slot_of[i] * fc.n_tiles);
                g_cnt.push_back(fc.n_tiles);
            }
        g_total += (int64_t)slot * fc.n_tiles;
        n_params += bc.n_params;
        psi_off[c] = state_total;
        const size_t sb = ((size_t)1 << n) * eb;
        state_total += (sb + 255) & ~(size_t)255;
        pass_bytes += 2.0 * (double)sb * (with_grad ? 3.0 * fc.n_pass + 1.0 : fc.n_pass + 0.5);
    }

    // ---- work segments, level-major: stage s of every circuit before stage s+1;
    //      inside a level forward stages, then observable stages, then reverse ----
    std::vector<FSeg> segs;
    int64_t n_items = 0;
    int max_stages = 0;
    std::vector<int> stages(n_circuits);
    for (int c = 0; c < n_circuits; ++c) {
        stages[c] = with_grad ? 2 * circs[c].n_pass + 1 : circs[c].n_pass + 1;
        max_stages = std::max(max_stages, stages[c]);
    }
    std::vector<int64_t> level_first;
    std::vector<uint8_t> level_gated(max_stages, 0);
    for (int s = 0; s < max_stages; ++s) {
        for (int kind = PM_FWD; kind <= PM_REV; ++kind) {
            level_first.push_back(n_items);
            for (int c = 0; c < n_circuits; ++c) {
                if (s >= stages[c]) continue;
                const int np = circs[c].n_pass;
                const int k = s < np ? PM_FWD : (s == np ? PM_OBS : PM_REV);
                if (k != kind) continue;
                if (k == PM_FWD && passes[circs[c].pass_begin + s].gated) level_gated[s] = 1;
                FSeg sg;
                sg.first = n_items;
                sg.circ = c;
                sg.stage = s;
                sg.n_tiles = circs[c].n_tiles;
                sg.pad = 0;
                segs.push_back(sg);
                n_items += circs[c].n_tiles;
            }
        }
    }
    level_first.push_back(n_items);
    if (n_items >= (1ll << 31)) return set_error(SV_ERR_UNSUPPORTED, "batch has too many work items");

    // ---- parameter -> slot CSR ----
    std::vector<int> csr_ptr(n_params + 1, 0), csr_col(slot_param.size());
    for (int p : slot_param) ++csr_ptr[p + 1];
    for (int j = 0; j < n_params; ++j) csr_ptr[j + 1] += csr_ptr[j];
    {
        std::vector<int> fill(csr_ptr.begin(), csr_ptr.end() - 1);
        for (size_t s = 0; s < slot_param.size(); ++s) csr_col[fill[slot_param[s]]++] = (int)s;
    }

    H.tq_max = tq_max;
    H.threads = pass_engine_threads(tq_used, reg_bits);
    H.rthreads = pass_engine_threads(tq_used, rreg_bits);
    if (H.threads > kMaxPassThreads || (with_grad && H.rthreads > kMaxPassThreads))
        return set_error(SV_ERR_ARG, "tile_qubits too large for amps_per_thread (at most 512 threads per tile)");
    H.reg_bits = reg_bits;
    H.rreg_bits = rreg_bits;
    H.n_levels = max_stages;
    H.lds_small = lds_small;
    H.with_grad = with_grad;
    H.cbits_default = cbits_default;
    H.n_params = n_params;
    H.coef_total = coef_total;
    H.tq_used = tq_used;
    H.hi_entries = hi_entries;
    H.e_total = e_total;
    H.g_total = g_total;
    H.n_items = n_items;
    H.state_total = state_total;
    H.pass_bytes = pass_bytes;
    H.circs = std::move(circs);
    H.passes = std::move(passes);
    H.fops = std::move(fops);
    H.lays = std::move(lays);
    H.cspec = std::move(cspec);
    H.cfac = std::move(cfac);
    H.slot_scale = std::move(slot_scale);
    H.slot_param = std::move(slot_param);
    H.g_off = std::move(g_off);
    H.e_off = std::move(e_off);
    H.level_first = std::move(level_first);
    H.level_gated = std::move(level_gated);
    H.g_cnt = std::move(g_cnt);
    H.e_cnt = std::move(e_cnt);
    H.csr_ptr = std::move(csr_ptr);
    H.csr_col = std::move(csr_col);
    H.segs = std::move(segs);
    H.psi_off = std::move(psi_off);
    H.n_gate_ops = 0;
    H.n_layout_changes = 0;
    for (const FPass& fp : H.passes)
        for (int o = fp.op_begin; o < fp.op_end; ++o) {
            if (H.fops[o].kind == FK_LAYOUT) ++H.n_layout_changes;
            else ++H.n_gate_ops;
        }
    return SV_OK;
}

// Largest dynamic LDS a workgroup of the batch uses (reverse passes hold the
// per-slot wave partials on top of the forward layout).
static size_t engine_lds_max(const HostTables& H, int dtype)
{
    return pass_engine_lds_bytes(H.tq_used, H.hi_entries, H.with_grad, dtype, H.lds_small,
                                 H.with_grad ? H.rthreads / 64 : 0);
}

sv_status sv_tune_engine_set(int dtype, int with_grad, int tile_qubits, int amps_per_thread)
{
    if (dtype != SV_C64 && dtype != SV_C128) return set_error(SV_ERR_ARG, "bad dtype");
    if (with_grad != 0 && with_grad != 1) return set_error(SV_ERR_ARG, "with_grad must be 0 or 1");
    if (amps_per_thread != 0 && amps_per_thread != 8 && amps_per_thread != 16)
        return set_error(SV_ERR_ARG, "amps_per_thread must be 0, 8 or 16");
    if (tile_qubits != 0 && (tile_qubits < 2 || tile_qubits > kMaxTileQubits))
        return set_error(SV_ERR_ARG, "tile_qubits must be 0 or in [2, 13]");
    if (tile_qubits) {
        const int rb = amps_per_thread == 8 ? 3 : 4;
        const int rrb = dtype == SV_C128 ? std::min(rb, 3) : rb;
        if (tile_qubits > engine_tq_fit(rb, rrb, with_grad))
            return set_error(SV_ERR_ARG, "tile_qubits too large for amps_per_thread (at most 512 threads per tile)");
    }
    const int d = dtype == SV_C128 ? 1 : 0;
    g_engine_tq[d][with_grad] = tile_qubits;
    g_engine_apt[d][with_grad] = amps_per_thread;
    return SV_OK;
}

sv_status sv_tune_engine_get(int dtype, int with_grad, int* tile_qubits, int* amps_per_thread)
{
    if ((dtype != SV_C64 && dtype != SV_C128) || (with_grad != 0 && with_grad != 1) || !tile_qubits ||
        !amps_per_thread)
        return set_error(SV_ERR_ARG, "bad dtype, with_grad or null output");
    const int d = dtype == SV_C128 ? 1 : 0;
    const int rb = g_engine_apt[d][with_grad] == 8 ? 3 : 4;
    const int rrb = dtype == SV_C128 ? std::min(rb, 3) : rb;
    const int tq_base = g_engine_tq[d][with_grad] > 0 ? g_engine_tq[d][with_grad] : (dtype == SV_C128 ? 12 : 13);
    *tile_qubits = std::min(tq_base, engine_tq_fit(rb, rrb, with_grad));
    *amps_per_thread = 1 << rb;
    return SV_OK;
}

sv_status sv_batch_plan(const sv_batch_circuit* circuits, int n_circuits, sv_dtype dtype, const sv_batch_opts* opts,
                        int64_t* info)
{
    if (!info) return set_error(SV_ERR_ARG, "null info");
    if (dtype != SV_C64 && dtype != SV_C128) return set_error(SV_ERR_ARG, "bad dtype");
    HostTables H;
    sv_status rc = compile_batch(circuits, n_circuits, dtype, opts, H);
    if (rc) return rc;
    int maxp = 0;
    for (const FCirc& c : H.circs) maxp = std::max(maxp, c.n_pass);
    info[0] = n_circuits;
    info[1] = H.n_items;
    info[2] = (int64_t)H.passes.size();
    info[3] = maxp;
    info[4] = H.n_gate_ops;
    info[5] = H.n_params;
    info[6] = (int64_t)H.state_total;
    info[7] = (int64_t)H.pass_bytes;
    info[8] = H.n_levels;
    info[9] = (int64_t)engine_lds_max(H, dtype);
    info[10] = H.n_layout_changes;
    info[11] = H.threads;
    return SV_OK;
}

sv_status sv_batch_create(const sv_batch_circuit* circuits, int n_circuits, sv_dtype dtype, const sv_batch_opts* opts,
                          sv_batch* out)
{
    if (!out) return set_error(SV_ERR_ARG, "null output handle");
    if (dtype != SV_C64 && dtype != SV_C128) return set_error(SV_ERR_ARG, "bad dtype");
    HostTables H;
    {
        sv_status rc = compile_batch(circuits, n_circuits, dtype, opts, H);
        if (rc) return rc;
    }
    const int with_grad = H.with_grad, threads = H.threads, n_params = H.n_params, coef_total = H.coef_total;
    const int tq_used = H.tq_used, hi_entries = H.hi_entries, e_total = H.e_total;
    const int64_t g_total = H.g_total, n_items = H.n_items;
    const size_t state_total = H.state_total;
    const double pass_bytes = H.pass_bytes;
    std::vector<FCirc>& circs = H.circs;
    std::vector<FPass>& passes = H.passes;
    std::vector<FOp>& fops = H.fops;
    std::vector<FCoefSpec>& cspec = H.cspec;
    std::vector<double>& slot_scale = H.slot_scale;
    std::vector<int>& slot_param = H.slot_param;
    std::vector<int64_t>& g_off = H.g_off;
    std::vector<int64_t>& e_off = H.e_off;
    std::vector<int64_t>& level_first = H.level_first;
    std::vector<int>& g_cnt = H.g_cnt;
    std::vector<int>& e_cnt = H.e_cnt;
    std::vector<int>& csr_ptr = H.csr_ptr;
    std::vector<int>& csr_col = H.csr_col;
    std::vector<FSeg>& segs = H.segs;
    std::vector<size_t>& psi_off = H.psi_off;
    // ---- device side ----
    sv_batch b = new sv_batch_s();
    b->dtype = dtype;
    b->n_circ = n_circuits;
    b->with_grad = with_grad;
    b->use_graph = opts ? (opts->use_graph != 0) : 1;
    b->threads = threads;
    b->rthreads = H.rthreads;
    b->reg_bits = H.reg_bits;
    b->rreg_bits = H.rreg_bits;
    b->n_levels = H.n_levels;
    b->n_items = n_items;
    b->n_segs = (int)segs.size();
    b->n_slots = (int)slot_param.size();
    b->n_params = n_params;
    b->n_passes = (int)passes.size();
    b->n_fops = H.n_gate_ops;
    b->n_layout_changes = H.n_layout_changes;
    b->state_bytes = state_total;
    b->pass_bytes = pass_bytes;
    b->psi_off = psi_off;
    b->n_cspec = (int)cspec.size();
    b->level_first = level_first;
    b->level_gated = H.level_gated;
    for (int c = 0; c < n_circuits; ++c) {
        b->nq.push_back(circs[c].n);
        b->max_passes = std::max(b->max_passes, circs[c].n_pass);
    }
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "stream");
    }
    b->caller = nullptr;
    e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_release(b);
        return hip_fail(e, "events");
    }
    if (hipMalloc(&b->d_psi, state_total) != hipSuccess ||
        (with_grad && hipMalloc(&b->d_lam, state_total) != hipSuccess)) {
        (void)hipGetLastError();
        batch_release(b);
        return set_error(SV_ERR_OOM, "batch state allocation failed");
    }
    for (int c = 0; c < n_circuits; ++c) {
        circs[c].psi = (char*)b->d_psi + psi_off[c];
        circs[c].lam = with_grad ? (char*)b->d_lam + psi_off[c] : nullptr;
    }
    std::vector<double> zeros_e(std::max(1, e_total)), zeros_p(std::max(1, n_params));
    e = dev_upload(&b->d_circ, circs);
    if (e == hipSuccess) e = dev_upload(&b->d_pass, passes);
    if (e == hipSuccess) e = dev_upload(&b->d_ops, fops);
    if (e == hipSuccess) e = dev_upload(&b->d_lays, H.lays);
    if (e == hipSuccess) e = dev_upload(&b->d_segs, segs);
    if (e == hipSuccess) e = dev_upload(&b->d_cspec, cspec);
    if (e == hipSuccess) e = dev_upload(&b->d_cfac, H.cfac);
    if (e == hipSuccess) e = dev_upload(&b->d_e_off, e_off);
    if (e == hipSuccess) e = dev_upload(&b->d_e_cnt, e_cnt);
    if (e == hipSuccess) e = dev_upload(&b->d_g_off, g_off);
    if (e == hipSuccess) e = dev_upload(&b->d_g_cnt, g_cnt);
    if (e == hipSuccess) e = dev_upload(&b->d_slot_scale, slot_scale);
    if (e == hipSuccess) e = dev_upload(&b->d_csr_ptr, csr_ptr);
    if (e == hipSuccess) e = dev_upload(&b->d_csr_col, csr_col);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_coef, sizeof(double) * std::max(1, coef_total));
    if (e == hipSuccess && dtype == SV_C64) e = hipMalloc((void**)&b->d_coef_f, sizeof(float) * std::max(1, coef_total));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_epart, sizeof(double) * std::max(1, e_total));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_gpart, sizeof(double) * std::max<int64_t>(1, g_total));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_slot_val, sizeof(double) * std::max<size_t>(1, slot_param.size()));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_params, sizeof(double) * std::max(1, n_params));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_expvals, sizeof(double) * n_circuits);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_grads, sizeof(double) * std::max(1, n_params));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        batch_release(b);
        return set_error(SV_ERR_OOM, "batch table allocation failed");
    }
    PassTables& tb = b->tb;
    tb.circs = b->d_circ;
    tb.passes = b->d_pass;
    tb.ops = b->d_ops;
    tb.lays = b->d_lays;
    tb.segs = b->d_segs;
    tb.coef = b->d_coef;
    tb.coef_f = b->d_coef_f;
    tb.e_part = b->d_epart;
    tb.g_part = b->d_gpart;
    tb.n_items = n_items;
    tb.n_segs = (int)segs.size();
    tb.tq_max = tq_used;
    tb.hi_entries = hi_entries;
    tb.with_grad = with_grad;
    tb.reg_bits = H.reg_bits;
    tb.rreg_bits = H.rreg_bits;
    tb.lds_small = H.lds_small;
    b->lds_fwd = pass_engine_lds_bytes(tq_used, hi_entries, with_grad, dtype, H.lds_small, 0);
    b->lds_rev = pass_engine_lds_bytes(tq_used, hi_entries, with_grad, dtype, H.lds_small, H.rthreads / 64);
    e = pass_engine_prepare(engine_lds_max(H, dtype));
    if (e != hipSuccess) {
        batch_release(b);
        return hip_fail(e, "pass engine LDS limit");
    }
    *out = (sv_batch)handle_put(b, HK_BATCH);
    return SV_OK;
}

#define SV_BATCH(b)                                                                    \
    sv_batch_s* const b = (sv_batch_s*)handle_get(b##_h, HK_BATCH);                     \
    if (!b) return set_error(SV_ERR_HANDLE, "invalid batch handle")

sv_status sv_batch_set_stream(sv_batch b_h, void* stream)
{
    SV_BATCH(b);
    b->caller = (hipStream_t)stream;
    return SV_OK;
}

sv_status sv_batch_run(sv_batch b_h, const double* params, int params_on_device, double* expvals, double* grads,
                       int outputs_on_device)
{
    SV_BATCH(b);
    if (b->n_params > 0 && !params) return set_error(SV_ERR_ARG, "null params");
    if (!expvals) return set_error(SV_ERR_ARG, "null expvals");
    if (b->with_grad && b->n_params > 0 && !grads) return set_error(SV_ERR_ARG, "null grads");
    hipStream_t s = b->stream;
    // start after the work already queued on the caller's stream (it may
    // still be writing the device-side parameters or clearing the outputs)
    hipError_t e = hipEventRecord(b->ev_in, b->caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_in, 0);
    if (e != hipSuccess) return hip_fail(e, "batch stream order");
    if (b->n_params > 0)
        e = hipMemcpyAsync(b->d_params, params, sizeof(double) * b->n_params,
                           params_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "batch params");
    if (b->use_graph) {
        if (!b->graph_ready) {
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "graph capture");
            hipError_t e2 = enqueue_run(b);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(s, &g);
            if (e2 != hipSuccess || e != hipSuccess) {
                // a failed capture leaves no graph behind: the next run captures again
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(e2 != hipSuccess ? e2 : e, e2 != hipSuccess ? "graph capture launch" : "graph end capture");
            }
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                b->exec = nullptr;
                return hip_fail(e, "graph instantiate");
            }
            b->graph = g;
            b->graph_ready = true;
        }
        e = hipGraphLaunch(b->exec, s);
    } else {
        e = enqueue_run(b);
    }
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    const hipMemcpyKind ok = outputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    e = hipMemcpyAsync(expvals, b->d_expvals, sizeof(double) * b->n_circ, ok, s);
    if (e == hipSuccess && b->with_grad && b->n_params > 0)
        e = hipMemcpyAsync(grads, b->d_grads, sizeof(double) * b->n_params, ok, s);
    // later work on the caller's stream sees the outputs
    if (e == hipSuccess) e = hipEventRecord(b->ev_out, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->caller, b->ev_out, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch run");
    return SV_OK;
}

sv_status sv_batch_info(sv_batch b_h, int64_t* info)
{
    SV_BATCH(b);
    if (!info) return set_error(SV_ERR_ARG, "null info");
    info[0] = b->n_circ;
    info[1] = b->n_items;
    info[2] = b->n_passes;
    info[3] = b->max_passes;
    info[4] = b->n_fops;
    info[5] = b->n_params;
    info[6] = (int64_t)b->state_bytes;
    info[7] = (int64_t)b->pass_bytes;
    info[8] = b->n_levels;
    info[9] = (int64_t)std::max(b->lds_fwd, b->with_grad ? b->lds_rev : 0);
    info[10] = b->n_layout_changes;
    info[11] = b->threads;
    return SV_OK;
}

sv_status sv_batch_state(sv_batch b_h, int circuit, void** dev_ptr, int* n_qubits)
{
    SV_BATCH(b);
    if (circuit < 0 || circuit >= b->n_circ || !dev_ptr) return set_error(SV_ERR_ARG, "bad circuit index");
    *dev_ptr = (char*)b->d_psi + b->psi_off[circuit];
    if (n_qubits) *n_qubits = b->nq[circuit];
    return SV_OK;
}

sv_status sv_batch_free(sv_batch b_h)
{
    sv_batch_s* const b = (sv_batch_s*)handle_drop(b_h, HK_BATCH);
    if (!b) return set_error(SV_ERR_HANDLE, "invalid batch handle");
    batch_release(b);
    return SV_OK;
}

sv_status sv_batch_copy_state(sv_batch b_h, int circuit, void* host, size_t bytes)
{
    SV_BATCH(b);
    if (circuit < 0 || circuit >= b->n_circ || !host) return set_error(SV_ERR_ARG, "bad circuit index or buffer");
    const size_t sb = ((size_t)1 << b->nq[circuit]) * (b->dtype == SV_C128 ? 16 : 8);
    if (bytes != sb) return set_error(SV_ERR_ARG, "byte count mismatch");
    hipError_t e = hipMemcpyAsync(host, (char*)b->d_psi + b->psi_off[circuit], sb, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return set_error(SV_ERR_HIP, std::string("batch state copy: ") + hipGetErrorString(e));
    return SV_OK;
}

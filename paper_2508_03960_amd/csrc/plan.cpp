// Subsequence classification and pass scheduling.  See plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace gbs {

static bool finite_all(const float *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

int validate_sequence(const gbs_block *blocks, int64_t n_blocks, int64_t total_steps,
                      const int32_t *adc_idx, int64_t total_samples, double dt, std::string &err) {
    if (n_blocks < 0 || total_steps < 0 || total_samples < 0) {
        err = "negative sequence size";
        return GBS_E_INVALID;
    }
    if (!(dt > 0.0) || !std::isfinite(dt)) {
        err = "dt must be positive and finite";
        return GBS_E_INVALID;
    }
    if (n_blocks > 0 && !blocks) {
        err = "blocks is null";
        return GBS_E_INVALID;
    }
    if (total_samples > 0 && !adc_idx) {
        err = "adc_idx is null";
        return GBS_E_INVALID;
    }
    for (int64_t b = 0; b < n_blocks; ++b) {
        const gbs_block &k = blocks[b];
        if (k.type == GBS_BLOCK_RELAX) {
            if (!(k.tau >= 0.0) || !std::isfinite(k.tau) || !std::isfinite(k.moment[0]) ||
                !std::isfinite(k.moment[1]) || !std::isfinite(k.moment[2])) {
                err = "relaxation block " + std::to_string(b) + ": bad tau or moment";
                return GBS_E_INVALID;
            }
            continue;
        }
        if (k.type != GBS_BLOCK_RF && k.type != GBS_BLOCK_ADC) {
            err = "block " + std::to_string(b) + ": unknown type";
            return GBS_E_INVALID;
        }
        if (k.n_steps < 0 || k.step_offset < 0 || k.step_offset + k.n_steps > total_steps ||
            k.n_steps > INT32_MAX) {
            err = "block " + std::to_string(b) + ": step range outside the waveform";
            return GBS_E_INVALID;
        }
        if (k.type == GBS_BLOCK_RF && k.n_samples != 0) {
            err = "RF block " + std::to_string(b) + " has samples (use an ADC block with B1)";
            return GBS_E_INVALID;
        }
        if (k.n_samples < 0 || k.sample_offset < 0 || k.sample_offset + k.n_samples > total_samples) {
            err = "block " + std::to_string(b) + ": sample range outside adc_idx";
            return GBS_E_INVALID;
        }
        for (int32_t n = 0; n < k.n_samples; ++n) {
            int32_t v = adc_idx[k.sample_offset + n];
            if (v < 0 || v > k.n_steps) {
                err = "block " + std::to_string(b) + ": ADC index outside its block";
                return GBS_E_INVALID;
            }
            if (n > 0 && v < adc_idx[k.sample_offset + n - 1]) {
                err = "block " + std::to_string(b) + ": ADC indices not in time order";
                return GBS_E_INVALID;
            }
        }
    }
    return GBS_OK;
}

void copy_sequence(HostSeq &s, const gbs_block *blocks, int64_t n_blocks, const float *rf_re,
                   const float *rf_im, const float *gx, const float *gy, const float *gz,
                   int64_t total_steps, const int32_t *adc_idx, int64_t total_samples, double dt) {
    s.blocks.assign(blocks, blocks + n_blocks);
    auto cp = [&](std::vector<float> &v, const float *p) {
        v.assign(total_steps, 0.0f);
        if (p && total_steps) std::memcpy(v.data(), p, sizeof(float) * total_steps);
    };
    cp(s.rf_re, rf_re);
    cp(s.rf_im, rf_im);
    cp(s.gx, gx);
    cp(s.gy, gy);
    cp(s.gz, gz);
    s.adc_idx.assign(adc_idx, adc_idx + total_samples);
    s.dt = dt;
    s.total_steps = total_steps;
    s.total_samples = total_samples;
    s.stepped_steps = 0;
    for (const auto &b : s.blocks)
        if (b.type != GBS_BLOCK_RELAX) s.stepped_steps += b.n_steps;
}

std::vector<BlockClass> classify(const HostSeq &s) {
    std::vector<BlockClass> out(s.blocks.size());
    for (size_t b = 0; b < s.blocks.size(); ++b) {
        const gbs_block &k = s.blocks[b];
        BlockClass &c = out[b];
        if (k.type == GBS_BLOCK_RELAX) continue;
        bool act[3] = {false, false, false};
        const std::vector<float> *g[3] = {&s.gx, &s.gy, &s.gz};
        for (int64_t j = k.step_offset; j < k.step_offset + k.n_steps; ++j) {
            if (s.rf_re[j] != 0.0f || s.rf_im[j] != 0.0f) c.has_b1 = true;
            for (int a = 0; a < 3; ++a) {
                float v = (*g[a])[j];
                if (v != 0.0f) act[a] = true;
                c.moment[a] += (double)v * s.dt;
            }
        }
        c.axes_mask = (act[0] ? 1 : 0) | (act[1] ? 2 : 0) | (act[2] ? 4 : 0);
        int na = act[0] + act[1] + act[2];
        if (na == 0)
            c.gtype = GT_NONE;
        else if (na > 1)
            c.gtype = GT_MIXED;
        else
            c.gtype = act[0] ? GT_X : (act[1] ? GT_Y : GT_Z);
    }
    return out;
}

// Split a stepped block into launches of at most max_samples samples.
static void add_step_ops(Plan &p, const HostSeq &s, int64_t b, const Map &pre, bool has_pre, int32_t max_samples) {
    const gbs_block &k = s.blocks[b];
    const int32_t ns = k.n_samples;
    if (ns == 0) {
        Op op;
        op.kind = 1;
        op.step = StepOp{b, has_pre, pre, 0, k.n_steps, 0, 0};
        p.ops.push_back(op);
        return;
    }
    for (int32_t a = 0; a < ns; a += max_samples) {
        int32_t e = std::min(ns, a + max_samples);
        Op op;
        op.kind = 1;
        op.step.block = b;
        op.step.has_pre = has_pre && a == 0;
        op.step.pre = a == 0 ? pre : Map{};
        op.step.step_lo = a == 0 ? 0 : s.adc_idx[k.sample_offset + a];
        op.step.step_hi = e == ns ? k.n_steps : s.adc_idx[k.sample_offset + e];
        op.step.sample_lo = a;
        op.step.sample_hi = e;
        p.ops.push_back(op);
    }
}

Plan plan_plain(const HostSeq &s, int32_t max_samples) {
    Plan p;
    Map P;
    for (size_t b = 0; b < s.blocks.size(); ++b) {
        const gbs_block &k = s.blocks[b];
        if (k.type == GBS_BLOCK_RELAX) {
            P.add(k.tau, k.moment);
            ++p.n_relax;
            continue;
        }
        add_step_ops(p, s, (int64_t)b, P, P.any(), max_samples);
        P = Map{};
    }
    if (P.any()) {
        Op op;
        op.kind = 1;
        op.step = StepOp{-1, true, P, 0, 0, 0, 0};
        p.ops.push_back(op);
    }
    return p;
}

static uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Index of the combined transition for RF block b applied per group of `axis`
// (-1: per isochromat); identical waveforms (B1 and all three gradients, bit
// for bit; the hash covers B1 and the active gradient) share one.
static int rf_lookup(Plan &p, std::vector<uint64_t> &hashes, const HostSeq &s, int64_t b, int axis,
                     int gtype) {
    const gbs_block &k = s.blocks[b];
    const std::vector<float> *g = gtype == GT_X ? &s.gx : gtype == GT_Y ? &s.gy : gtype == GT_Z ? &s.gz : nullptr;
    const size_t nb = sizeof(float) * (size_t)k.n_steps;
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &axis, sizeof(axis));
    h = fnv1a(h, &k.n_steps, sizeof(k.n_steps));
    h = fnv1a(h, s.rf_re.data() + k.step_offset, nb);
    h = fnv1a(h, s.rf_im.data() + k.step_offset, nb);
    if (g) h = fnv1a(h, g->data() + k.step_offset, nb);
    for (size_t i = 0; i < p.rf.size(); ++i) {
        const RfJob &r = p.rf[i];
        if (hashes[i] != h || r.axis != axis || r.n_steps != k.n_steps) continue;
        bool same = !std::memcmp(s.rf_re.data() + k.step_offset, s.rf_re.data() + r.step_offset, nb) &&
                    !std::memcmp(s.rf_im.data() + k.step_offset, s.rf_im.data() + r.step_offset, nb);
        for (int a = 0; a < 3 && same; ++a) {
            const std::vector<float> &ga = a == 0 ? s.gx : a == 1 ? s.gy : s.gz;
            same = !std::memcmp(ga.data() + k.step_offset, ga.data() + r.step_offset, nb);
        }
        if (same) return (int)i;
    }
    p.rf.push_back(RfJob{axis, k.step_offset, k.n_steps});
    hashes.push_back(h);
    return (int)p.rf.size() - 1;
}

Plan plan_grouped(const HostSeq &s, const std::vector<BlockClass> &cls, uint32_t axes_built, int32_t max_samples) {
    Plan p;
    std::vector<uint64_t> hashes;
    Map P;  // B1 = 0 maps since the state in memory (or the pending pass) was last advanced
    bool have_cur = false;
    PassOp cur;
    auto flush = [&]() {
        if (!have_cur) return;
        Op op;
        op.kind = 0;
        op.pass = cur;
        p.ops.push_back(op);
        ++p.n_passes;
        have_cur = false;
    };
    for (size_t bi = 0; bi < s.blocks.size(); ++bi) {
        const int64_t b = (int64_t)bi;
        const gbs_block &k = s.blocks[bi];
        const BlockClass &c = cls[bi];
        if (k.type == GBS_BLOCK_RELAX) {
            P.add(k.tau, k.moment);
            ++p.n_relax;
            continue;
        }
        const double dur = (double)k.n_steps * s.dt;
        if (k.type == GBS_BLOCK_RF && !c.has_b1) {
            // B1 = 0 over the block: the stepped product equals the closed form.
            P.add(dur, c.moment);
            ++p.n_b1zero;
            continue;
        }
        const int axis = c.gtype == GT_NONE ? GT_X : c.gtype;
        const bool known = c.gtype != GT_MIXED && (axes_built & (1u << axis));
        if (k.type == GBS_BLOCK_RF && c.gtype == GT_MIXED && c.axes_mask == 5 && (axes_built & GBS_AX_XZ)) {
            // Gx and Gz together (an oblique slice): one transition per (x, z) group
            flush();
            cur = PassOp{};
            cur.has_pre = P.any();
            cur.pre = P;
            cur.rf_axis = kPairRows;
            cur.rf_id = rf_lookup(p, hashes, s, b, kPairAxis, c.gtype);
            cur.write_m = true;
            have_cur = true;
            P = Map{};
            ++p.n_rf_grouped;
            continue;
        }
        if (k.type == GBS_BLOCK_RF && known) {
            flush();
            cur = PassOp{};
            cur.has_pre = P.any();
            cur.pre = P;
            cur.rf_axis = axis;
            // no-grads: one composition per tissue group when those exist (the
            // sweep still applies it through the x-group rows)
            const int job_axis = c.gtype == GT_NONE && (axes_built & GBS_AX_N) ? kTissueAxis : axis;
            cur.rf_id = rf_lookup(p, hashes, s, b, job_axis, c.gtype);
            cur.write_m = true;
            have_cur = true;
            P = Map{};
            ++p.n_rf_grouped;
            continue;
        }
        if (k.type == GBS_BLOCK_ADC && !c.has_b1 && known) {
            const int job = (int)p.adc.size();
            p.adc.push_back(AdcJob{axis, b});
            if (have_cur) {
                cur.emit_axis = axis;
                cur.emit = P;
                cur.adc_job = job;
                flush();
            } else {
                Op op;
                op.kind = 0;
                op.pass.has_pre = false;
                op.pass.write_m = false;
                op.pass.emit_axis = axis;
                op.pass.emit = P;
                op.pass.adc_job = job;
                p.ops.push_back(op);
                ++p.n_passes;
                ++p.n_emit_only;
            }
            P.add(dur, c.moment);  // third step: members to the block end by Eq. (4), (5)
            ++p.n_adc_grouped;
            continue;
        }
        // Unclassified, RF together with ADC, or an axis without groups:
        // the conventional per-isochromat stepping (Sec. 3.1).
        flush();
        add_step_ops(p, s, b, P, P.any(), max_samples);
        P = Map{};
        ++p.n_fallback;
    }
    flush();
    p.final_pass = P.any();
    p.final_map = P;
    return p;
}

Plan plan_cached(const HostSeq &s, const std::vector<BlockClass> &cls, int32_t max_samples) {
    Plan p;
    std::vector<uint64_t> hashes;
    Map P;  // B1 = 0 maps not yet applied to the stored state
    for (size_t bi = 0; bi < s.blocks.size(); ++bi) {
        const int64_t b = (int64_t)bi;
        const gbs_block &k = s.blocks[bi];
        const BlockClass &c = cls[bi];
        if (k.type == GBS_BLOCK_RELAX) {
            P.add(k.tau, k.moment);
            ++p.n_relax;
            continue;
        }
        const double dur = (double)k.n_steps * s.dt;
        if (!c.has_b1) {
            if (k.type == GBS_BLOCK_RF) {
                ++p.n_b1zero;
            } else {
                // static isochromats, no RF: every sample from the block-start state
                for (int32_t a = 0; a < k.n_samples; a += kMaxSamplesPerLaunch) {
                    Op op;
                    op.kind = 3;
                    op.cached.block = b;
                    op.cached.has_pre = P.any();
                    op.cached.pre = P;
                    op.cached.sample_lo = a;
                    op.cached.sample_hi = std::min(k.n_samples, a + kMaxSamplesPerLaunch);
                    p.ops.push_back(op);
                }
                ++p.n_adc_direct;
            }
            P.add(dur, c.moment);
            continue;
        }
        if (k.type == GBS_BLOCK_RF) {
            const size_t before = p.rf.size();
            Op op;
            op.kind = 2;
            op.cached.block = b;
            op.cached.has_pre = P.any();
            op.cached.pre = P;
            op.cached.entry = rf_lookup(p, hashes, s, b, -1, GT_MIXED);
            op.cached.compose = p.rf.size() > before;
            p.ops.push_back(op);
            P = Map{};
            ++p.n_rf_cached;
            continue;
        }
        // RF during an ADC block: stepped per isochromat
        add_step_ops(p, s, b, P, P.any(), max_samples);
        P = Map{};
        ++p.n_fallback;
    }
    Op op;
    op.kind = 4;
    op.cached.has_pre = P.any();
    op.cached.pre = P;
    p.ops.push_back(op);
    return p;
}

}  // namespace gbs

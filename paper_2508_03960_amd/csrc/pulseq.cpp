// Pulseq sequence files (format 1.4) rasterized into the block sequence the
// simulator runs (Sec. 2.1, Fig. 1): a Pulseq block is one subsequence,
// classified by the events it holds -- with-RF, with-ADC (RF during ADC is
// kept as a with-ADC subsequence), or relaxation -- and its waveforms are
// sampled on the simulator's uniform raster dt.
//
// Event semantics taken from the Pulseq format:
//   * RF: complex amplitude amp * mag_i * exp(i (phase + 2 pi ph_i)), sample i
//     held over [delay + i d_rf, delay + (i + 1) d_rf) (d_rf = the RF raster);
//     a frequency offset adds 2 pi f t at the sample centre t, counted from
//     the event start;
//   * trapezoid: 0 -> amp over `rise`, flat, amp -> 0 over `fall`, after
//     `delay`;
//   * arbitrary gradient: piecewise linear through its points -- on the
//     default timing (first, then sample i at (i + 0.5) d_g, then last at
//     n d_g), or at the times of its time shape (units of d_g);
//   * ADC: sample j at delay + (j + 0.5) dwell from the block start;
//   * shapes: the compressed form (run-length coded derivative) unless the
//     listed values number num_samples.
// Each raster step holds the exact average of the waveform over the step,
// so gradient moments and RF areas are kept exactly.  Hz and Hz/m become
// tesla and T/m through gamma / 2 pi.
#include <algorithm>
#include <cctype>
#include <cerrno>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "consts.hpp"
#include "gbloch.h"

namespace {

// Limits on what one file may ask for: stepped raster steps and ADC samples
// (2^28: 268 s of RF and ADC time on a 1 us raster, about 5.4 GB of
// waveforms) and samples of one shape.
constexpr int64_t kMaxSteps = int64_t(1) << 28;
constexpr int64_t kMaxSamples = int64_t(1) << 28;
constexpr long kMaxShape = 1L << 26;

struct Fail {
    std::string msg;
};

[[noreturn]] void fail(const std::string &m) { throw Fail{m}; }

struct RfEv {
    double amp;  // Hz
    long mag, phase, time;
    double delay_us, freq, phase_off;
};
struct GradEv {
    double amp, first, last;  // Hz/m
    long shape, time;
    double delay_us;
};
struct TrapEv {
    double amp;  // Hz/m
    double rise, flat, fall, delay;  // us
};
struct AdcEv {
    long num;
    double dwell_ns, delay_us, freq, phase;
};
struct BlockRow {
    long num, dur, rf, g[3], adc;
};

struct File {
    long major = -1, minor = -1;
    double grad_raster = 10e-6, rf_raster = 1e-6, adc_raster = 100e-9, block_raster = 10e-6;
    std::vector<BlockRow> blocks;
    std::map<long, RfEv> rf;
    std::map<long, GradEv> grad;
    std::map<long, TrapEv> trap;
    std::map<long, AdcEv> adc;
    std::map<long, std::vector<double>> shapes;
};

std::vector<std::string> tokens(const std::string &line) {
    std::vector<std::string> t;
    size_t i = 0, n = line.size();
    while (i < n) {
        while (i < n && std::isspace((unsigned char)line[i])) ++i;
        size_t j = i;
        while (j < n && !std::isspace((unsigned char)line[j])) ++j;
        if (j > i) t.push_back(line.substr(i, j - i));
        i = j;
    }
    return t;
}

double num(const std::string &s, long line) {
    char *end = nullptr;
    double v = std::strtod(s.c_str(), &end);
    if (end == s.c_str() || *end != '\0' || !std::isfinite(v))
        fail("line " + std::to_string(line) + ": '" + s + "' is not a finite number");
    return v;
}

long inum(const std::string &s, long line) {
    char *end = nullptr;
    errno = 0;
    long v = std::strtol(s.c_str(), &end, 10);
    if (end == s.c_str() || *end != '\0' || errno == ERANGE || v > INT32_MAX || v < INT32_MIN)
        fail("line " + std::to_string(line) + ": '" + s + "' is not a 32-bit integer");
    return v;
}

void need(const std::vector<std::string> &t, size_t n, const char *sec, long line) {
    if (t.size() != n)
        fail("line " + std::to_string(line) + ": [" + sec + "] rows have " + std::to_string(n) + " columns in format 1.4, found " +
             std::to_string(t.size()));
}

// The compressed shape form: the derivative of the samples with runs coded as
// (v, v, r) = r + 2 copies of v; the samples are its running sum.
std::vector<double> decode_shape(const std::vector<double> &packed, long n_samples, long id) {
    if ((long)packed.size() == n_samples) return packed;
    std::vector<double> d;
    size_t i = 0;
    while (i < packed.size()) {
        if (i + 1 < packed.size() && packed[i] == packed[i + 1]) {
            if (i + 2 >= packed.size()) fail("shape " + std::to_string(id) + ": run without a count");
            double r = packed[i + 2];
            if (r < 0 || r != std::floor(r)) fail("shape " + std::to_string(id) + ": bad run count");
            if ((double)d.size() + r + 2 > (double)n_samples)
                fail("shape " + std::to_string(id) + ": decodes to more than num_samples = " + std::to_string(n_samples));
            d.insert(d.end(), (size_t)r + 2, packed[i]);
            i += 3;
        } else {
            d.push_back(packed[i]);
            i += 1;
        }
    }
    if ((long)d.size() != n_samples)
        fail("shape " + std::to_string(id) + ": decodes to " + std::to_string(d.size()) + " samples, num_samples is " +
             std::to_string(n_samples));
    double s = 0.0;
    for (double &v : d) {
        s += v;
        v = s;
    }
    return d;
}

File parse(const char *text, int64_t len) {
    File f;
    std::string sec;
    long shape_id = -1, shape_n = -1;
    std::vector<double> packed;
    std::map<long, std::pair<long, std::vector<double>>> raw_shapes;
    auto close_shape = [&]() {
        if (shape_id < 0) return;
        if (shape_n < 0) fail("shape " + std::to_string(shape_id) + ": no num_samples");
        if (raw_shapes.count(shape_id)) fail("shape " + std::to_string(shape_id) + " defined twice");
        raw_shapes[shape_id] = {shape_n, packed};
        shape_id = shape_n = -1;
        packed.clear();
    };
    int64_t pos = 0;
    long line_no = 0;
    while (pos < len) {
        int64_t e = pos;
        while (e < len && text[e] != '\n') ++e;
        std::string line(text + pos, text + e);
        pos = e + 1;
        ++line_no;
        size_t h = line.find('#');
        if (h != std::string::npos) line.resize(h);
        auto t = tokens(line);
        if (t.empty()) continue;
        if (t[0].front() == '[') {
            close_shape();
            sec = t[0];
            continue;
        }
        if (sec == "[VERSION]") {
            if (t.size() != 2) fail("line " + std::to_string(line_no) + ": bad [VERSION] row");
            if (t[0] == "major") f.major = inum(t[1], line_no);
            if (t[0] == "minor") f.minor = inum(t[1], line_no);
        } else if (sec == "[DEFINITIONS]") {
            if (t.size() < 2) continue;
            if (t[0] == "GradientRasterTime") f.grad_raster = num(t[1], line_no);
            if (t[0] == "RadiofrequencyRasterTime") f.rf_raster = num(t[1], line_no);
            if (t[0] == "AdcRasterTime") f.adc_raster = num(t[1], line_no);
            if (t[0] == "BlockDurationRaster") f.block_raster = num(t[1], line_no);
        } else if (sec == "[BLOCKS]") {
            need(t, 8, "BLOCKS", line_no);
            BlockRow b{inum(t[0], line_no), inum(t[1], line_no), inum(t[2], line_no),
                       {inum(t[3], line_no), inum(t[4], line_no), inum(t[5], line_no)}, inum(t[6], line_no)};
            if (b.dur < 0) fail("line " + std::to_string(line_no) + ": negative block duration");
            f.blocks.push_back(b);
        } else if (sec == "[RF]") {
            need(t, 8, "RF", line_no);
            long id = inum(t[0], line_no);
            f.rf[id] = RfEv{num(t[1], line_no),      inum(t[2], line_no),     inum(t[3], line_no), inum(t[4], line_no),
                            num(t[5], line_no),      num(t[6], line_no),      num(t[7], line_no)};
        } else if (sec == "[GRADIENTS]") {
            need(t, 7, "GRADIENTS", line_no);
            long id = inum(t[0], line_no);
            f.grad[id] = GradEv{num(t[1], line_no), num(t[2], line_no), num(t[3], line_no), inum(t[4], line_no),
                                inum(t[5], line_no), num(t[6], line_no)};
        } else if (sec == "[TRAP]") {
            need(t, 6, "TRAP", line_no);
            long id = inum(t[0], line_no);
            f.trap[id] = TrapEv{num(t[1], line_no), num(t[2], line_no), num(t[3], line_no), num(t[4], line_no),
                                num(t[5], line_no)};
        } else if (sec == "[ADC]") {
            need(t, 6, "ADC", line_no);
            long id = inum(t[0], line_no);
            f.adc[id] = AdcEv{inum(t[1], line_no), num(t[2], line_no), num(t[3], line_no), num(t[4], line_no),
                              num(t[5], line_no)};
        } else if (sec == "[SHAPES]") {
            if (t[0] == "shape_id") {
                close_shape();
                if (t.size() != 2) fail("line " + std::to_string(line_no) + ": bad shape_id row");
                shape_id = inum(t[1], line_no);
            } else if (t[0] == "num_samples") {
                if (t.size() != 2 || shape_id < 0) fail("line " + std::to_string(line_no) + ": bad num_samples row");
                shape_n = inum(t[1], line_no);
                if (shape_n < 1 || shape_n > kMaxShape)
                    fail("line " + std::to_string(line_no) + ": num_samples outside [1, 2^26]");
            } else {
                if (shape_id < 0 || shape_n < 0) fail("line " + std::to_string(line_no) + ": shape values before shape_id/num_samples");
                for (auto &s : t) packed.push_back(num(s, line_no));
            }
        }
        // [EXTENSIONS], [SIGNATURE] and unknown sections carry nothing the
        // simulation uses.
    }
    close_shape();
    if (f.major < 0 || f.minor < 0) fail("no [VERSION] section with major and minor");
    if (f.major != 1 || f.minor != 4)
        fail("Pulseq format version " + std::to_string(f.major) + "." + std::to_string(f.minor) +
             " is not supported (format 1.4 only)");
    for (double r : {f.grad_raster, f.rf_raster, f.adc_raster, f.block_raster})
        if (!(r > 0)) fail("raster times must be > 0");
    for (auto &kv : raw_shapes) f.shapes[kv.first] = decode_shape(kv.second.second, kv.second.first, kv.first);
    return f;
}

const std::vector<double> &shape(const File &f, long id, const char *what) {
    auto it = f.shapes.find(id);
    if (it == f.shapes.end()) fail(std::string(what) + " refers to missing shape " + std::to_string(id));
    return it->second;
}

// Piecewise-linear waveform (seconds from the block start, T/m).
struct Pts {
    std::vector<double> t, v;
    void add(double tt, double vv) {
        if (!t.empty() && tt < t.back() - 1e-15) fail("gradient time points decrease");
        t.push_back(tt);
        v.push_back(vv);
    }
    double end() const { return t.empty() ? 0.0 : t.back(); }
};

Pts gradient_points(const File &f, long id, char axis) {
    Pts p;
    const std::string name = std::string("G") + axis;
    if (f.trap.count(id) && f.grad.count(id)) fail(name + " id " + std::to_string(id) + " is both [TRAP] and [GRADIENTS]");
    auto tr = f.trap.find(id);
    if (tr != f.trap.end()) {
        const TrapEv &e = tr->second;
        if (e.rise < 0 || e.flat < 0 || e.fall < 0 || e.delay < 0) fail("trapezoid " + std::to_string(id) + ": negative time");
        double a = e.amp / gbs::kGammaBar, t0 = e.delay * 1e-6;
        p.add(t0, 0.0);
        p.add(t0 + e.rise * 1e-6, a);
        p.add(t0 + (e.rise + e.flat) * 1e-6, a);
        p.add(t0 + (e.rise + e.flat + e.fall) * 1e-6, 0.0);
        return p;
    }
    auto gr = f.grad.find(id);
    if (gr == f.grad.end()) fail(name + " refers to missing gradient " + std::to_string(id));
    const GradEv &e = gr->second;
    if (e.delay_us < 0) fail("gradient " + std::to_string(id) + ": negative delay");
    const std::vector<double> &s = shape(f, e.shape, "gradient");
    double a = e.amp / gbs::kGammaBar, t0 = e.delay_us * 1e-6, d = f.grad_raster;
    if (e.time == 0) {
        p.add(t0, e.first / gbs::kGammaBar);
        for (size_t i = 0; i < s.size(); ++i) p.add(t0 + (i + 0.5) * d, a * s[i]);
        p.add(t0 + s.size() * d, e.last / gbs::kGammaBar);
    } else {
        const std::vector<double> &ts = shape(f, e.time, "gradient time");
        if (ts.size() != s.size()) fail("gradient " + std::to_string(id) + ": time and amplitude shapes differ in length");
        for (size_t i = 0; i < s.size(); ++i) p.add(t0 + ts[i] * d, a * s[i]);
    }
    return p;
}

// Adds the integral of the waveform over every raster step [j dt, (j+1) dt)
// to acc[j] (acc has n entries) and returns the total integral.
double integrate_linear(const Pts &p, double dt, double *acc, int64_t n) {
    double total = 0.0;
    for (size_t k = 0; k + 1 < p.t.size(); ++k) {
        double t0 = p.t[k], t1 = p.t[k + 1], v0 = p.v[k], v1 = p.v[k + 1];
        if (!(t1 > t0)) continue;
        double slope = (v1 - v0) / (t1 - t0);
        total += 0.5 * (v0 + v1) * (t1 - t0);
        if (!acc) continue;
        int64_t j0 = (int64_t)std::floor(t0 / dt), j1 = (int64_t)std::ceil(t1 / dt);
        for (int64_t j = std::max<int64_t>(j0, 0); j < std::min(j1, n); ++j) {
            double u0 = std::max(t0, j * dt), u1 = std::min(t1, (j + 1) * dt);
            if (u1 <= u0) continue;
            acc[j] += 0.5 * ((v0 + slope * (u0 - t0)) + (v0 + slope * (u1 - t0))) * (u1 - u0);
        }
    }
    return total;
}

float to_float(double v, const char *what) {
    float f = (float)v;
    if (!std::isfinite(f)) fail(std::string(what) + " value outside the float range");
    return f;
}

struct Out {
    std::vector<gbs_block> blocks;
    std::vector<float> rf_re, rf_im, g[3];
    std::vector<int32_t> adc_idx;
    std::vector<double> adc_phase;
};

void rasterize(const File &f, double dt, bool fill, Out &o, int64_t &steps, int64_t &samples) {
    const double tol = 1e-9;  // s: events may end this far past their block
    steps = samples = 0;
    for (const BlockRow &b : f.blocks) {
        const std::string at = "block " + std::to_string(b.num) + ": ";
        double D = b.dur * f.block_raster;
        bool has_rf = b.rf != 0, has_adc = b.adc != 0;
        bool has_g = b.g[0] != 0 || b.g[1] != 0 || b.g[2] != 0;
        if (D == 0.0) {
            if (has_rf || has_adc || has_g) fail(at + "events in a block of zero duration");
            continue;  // a label-only block
        }
        // only stepped blocks live on the raster; a relaxation block keeps
        // its exact duration
        int64_t n = 0;
        if (has_rf || has_adc) {
            double q = D / dt;
            if (!(q <= (double)kMaxSteps)) fail(at + "longer than 2^28 raster steps");
            n = (int64_t)std::llround(q);
            if (n == 0 || std::fabs(q - n) > 1e-6 * std::max<double>(1.0, n))
                fail(at + "duration " + std::to_string(D) + " s is not a whole number of raster steps dt");
        }
        Pts gp[3];
        for (int a = 0; a < 3; ++a) {
            if (!b.g[a]) continue;
            gp[a] = gradient_points(f, b.g[a], "xyz"[a]);
            if (gp[a].end() > D + tol) fail(at + "gradient on axis " + std::string(1, "xyz"[a]) + " outlasts the block");
        }
        gbs_block blk{};
        if (!has_rf && !has_adc) {
            blk.type = GBS_BLOCK_RELAX;
            blk.tau = D;
            for (int a = 0; a < 3; ++a) {
                blk.moment[a] = b.g[a] ? integrate_linear(gp[a], dt, nullptr, 0) : 0.0;
                if (!std::isfinite(blk.moment[a])) fail(at + "gradient moment is not finite");
            }
            blk.step_offset = steps;
            blk.sample_offset = samples;
            o.blocks.push_back(blk);
            continue;
        }
        if (steps + n > kMaxSteps) fail("more than 2^28 stepped raster steps");
        blk.type = has_adc ? GBS_BLOCK_ADC : GBS_BLOCK_RF;
        blk.step_offset = steps;
        blk.n_steps = n;
        blk.sample_offset = samples;
        if (has_adc) {
            auto it = f.adc.find(b.adc);
            if (it == f.adc.end()) fail(at + "missing ADC event " + std::to_string(b.adc));
            const AdcEv &e = it->second;
            if (e.num < 0 || e.dwell_ns <= 0 || e.delay_us < 0) fail(at + "bad ADC event");
            // samples lie on distinct boundaries 0..n
            if (e.num > n + 1) fail(at + "ADC samples outlast the block");
            if (samples + e.num > kMaxSamples) fail("more than 2^28 ADC samples");
            for (long j = 0; j < e.num; ++j) {
                double t = e.delay_us * 1e-6 + (j + 0.5) * e.dwell_ns * 1e-9;
                double r = t / dt;
                if (!(r <= n + 0.5)) fail(at + "ADC samples outlast the block");
                int64_t k = (int64_t)std::llround(r);
                if (std::fabs(r - k) > 1e-6 * std::max<double>(1.0, k))
                    fail(at + "ADC sample " + std::to_string(j) + " at " + std::to_string(t) +
                         " s is not on a raster boundary (choose dt dividing the sample times)");
                if (k > n) fail(at + "ADC samples outlast the block");
                if (fill) {
                    o.adc_idx.push_back((int32_t)k);
                    o.adc_phase.push_back(e.phase + 2.0 * M_PI * e.freq * (t - e.delay_us * 1e-6));
                }
            }
            blk.n_samples = (int32_t)e.num;
            samples += e.num;
        }
        if (fill) {
            std::vector<double> acc(n), re(n, 0.0), im(n, 0.0);
            for (int a = 0; a < 3; ++a) {
                std::fill(acc.begin(), acc.end(), 0.0);
                if (b.g[a]) integrate_linear(gp[a], dt, acc.data(), n);
                for (int64_t j = 0; j < n; ++j) o.g[a].push_back(to_float(acc[j] / dt, "gradient"));
            }
            if (has_rf) {
                auto it = f.rf.find(b.rf);
                if (it == f.rf.end()) fail(at + "missing RF event " + std::to_string(b.rf));
                const RfEv &e = it->second;
                if (e.time != 0) fail(at + "RF events with a time shape are not supported (default RF raster only)");
                if (e.delay_us < 0) fail(at + "negative RF delay");
                const std::vector<double> &mag = shape(f, e.mag, "RF magnitude");
                const std::vector<double> *ph = e.phase ? &shape(f, e.phase, "RF phase") : nullptr;
                if (ph && ph->size() != mag.size()) fail(at + "RF magnitude and phase shapes differ in length");
                double d = f.rf_raster, t0 = e.delay_us * 1e-6;
                if (t0 + mag.size() * d > D + tol) fail(at + "RF outlasts the block");
                double amp = e.amp / gbs::kGammaBar;
                for (size_t i = 0; i < mag.size(); ++i) {
                    double phi = e.phase_off + (ph ? 2.0 * M_PI * (*ph)[i] : 0.0) + 2.0 * M_PI * e.freq * (i + 0.5) * d;
                    double cr = amp * mag[i] * std::cos(phi), ci = amp * mag[i] * std::sin(phi);
                    double s0 = t0 + i * d, s1 = s0 + d;
                    int64_t j0 = std::max<int64_t>((int64_t)std::floor(s0 / dt), 0);
                    int64_t j1 = std::min<int64_t>((int64_t)std::ceil(s1 / dt), n);
                    for (int64_t j = j0; j < j1; ++j) {
                        double w = std::min(s1, (j + 1) * dt) - std::max(s0, j * dt);
                        if (w <= 0) continue;
                        re[j] += cr * w;
                        im[j] += ci * w;
                    }
                }
            }
            for (int64_t j = 0; j < n; ++j) {
                o.rf_re.push_back(to_float(re[j] / dt, "RF"));
                o.rf_im.push_back(to_float(im[j] / dt, "RF"));
            }
            o.blocks.push_back(blk);
        } else {
            if (has_rf) {
                auto it = f.rf.find(b.rf);
                if (it == f.rf.end()) fail(at + "missing RF event " + std::to_string(b.rf));
            }
            o.blocks.emplace_back();
        }
        steps += n;
    }
}

void put_err(char *err, int64_t cap, const std::string &m) {
    if (!err || cap <= 0) return;
    size_t k = std::min<size_t>(m.size(), (size_t)cap - 1);
    std::memcpy(err, m.data(), k);
    err[k] = '\0';
}

}  // namespace

extern "C" int gbs_pulseq_load(const char *text, int64_t text_len, double dt, int64_t sizes[3], gbs_block *blocks,
                               float *rf_re, float *rf_im, float *gx, float *gy, float *gz, int32_t *adc_idx,
                               double *adc_phase, double rasters[4], char *err, int64_t err_cap) {
    put_err(err, err_cap, "");
    if (!text || text_len < 0 || !sizes) {
        put_err(err, err_cap, "text and sizes must not be null");
        return GBS_E_INVALID;
    }
    try {
        File f = parse(text, text_len);
        if (rasters) {
            rasters[0] = f.grad_raster;
            rasters[1] = f.rf_raster;
            rasters[2] = f.adc_raster;
            rasters[3] = f.block_raster;
        }
        if (!(dt > 0)) dt = f.rf_raster;
        if (!std::isfinite(dt)) fail("dt must be finite");
        const bool fill = blocks != nullptr;
        int64_t cap[3] = {sizes[0], sizes[1], sizes[2]};
        Out o;
        int64_t steps = 0, samples = 0;
        rasterize(f, dt, fill, o, steps, samples);
        sizes[0] = (int64_t)o.blocks.size();
        sizes[1] = steps;
        sizes[2] = samples;
        if (!fill) return GBS_OK;
        if (sizes[0] > cap[0] || sizes[1] > cap[1] || sizes[2] > cap[2])
            fail("output buffers smaller than the sizes of the sequence");
        if ((steps > 0 && (!rf_re || !rf_im || !gx || !gy || !gz)) || (samples > 0 && !adc_idx))
            fail("a needed output buffer is null");
        if (!o.blocks.empty()) std::memcpy(blocks, o.blocks.data(), o.blocks.size() * sizeof(gbs_block));
        if (steps > 0) {
            std::memcpy(rf_re, o.rf_re.data(), steps * sizeof(float));
            std::memcpy(rf_im, o.rf_im.data(), steps * sizeof(float));
            std::memcpy(gx, o.g[0].data(), steps * sizeof(float));
            std::memcpy(gy, o.g[1].data(), steps * sizeof(float));
            std::memcpy(gz, o.g[2].data(), steps * sizeof(float));
        }
        if (samples > 0) {
            std::memcpy(adc_idx, o.adc_idx.data(), samples * sizeof(int32_t));
            if (adc_phase) std::memcpy(adc_phase, o.adc_phase.data(), samples * sizeof(double));
        }
        return GBS_OK;
    } catch (const Fail &e) {
        put_err(err, err_cap, e.msg);
        return GBS_E_INVALID;
    } catch (const std::bad_alloc &) {
        put_err(err, err_cap, "out of host memory");
        return GBS_E_NOMEM;
    }
}

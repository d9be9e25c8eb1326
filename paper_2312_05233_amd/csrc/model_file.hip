// Model files: a plain-text form of tnep_model_desc (every parameter of the
// descriptor and of the networks of Sec. 2.1, Eq. site-energy), written with
// 17 significant digits so that FP64 values survive the round trip exactly.
//
//   tnep_model 1
//   kind dipole|polarizability|pes
//   n_species T
//   rc <rc_radial> <rc_angular>
//   n_max <nR> <nA>
//   basis <KR> <KA>
//   l_max 4
//   four_body 0|1
//   five_body 0|1
//   n_hidden H
//   per_species 0|1
//   c_radial   T*T*(nR+1)*(KR+1) numbers
//   c_angular  T*T*(nA+1)*(KA+1) numbers
//   q_scaler   D numbers
//   head <h>   (h = 0, and h = 1 for polarizability models), then
//     w0 NS*H*D numbers   b0 NS*H   w1 NS*H   b1 NS   (NS = T if per_species else 1)
//   end
//
// Tokens are separated by white space; '#' starts a comment to the end of the line.
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

using namespace tnep;

namespace {

int descriptor_length(const tnep_model_desc& d) {
    const int na = d.n_max_angular + 1;
    return d.n_max_radial + 1 + d.l_max * na + (d.four_body ? na : 0) + (d.five_body ? na : 0);
}

const char* kind_name(int k) {
    return k == TNEP_KIND_DIPOLE ? "dipole" : k == TNEP_KIND_POLARIZABILITY ? "polarizability" : "pes";
}

struct Reader {
    std::string text;
    size_t pos = 0;
    int line = 1;
    std::string err;

    bool next(std::string& tok) {
        for (;;) {
            while (pos < text.size() && isspace((unsigned char)text[pos])) {
                if (text[pos] == '\n') ++line;
                ++pos;
            }
            if (pos < text.size() && text[pos] == '#') {
                while (pos < text.size() && text[pos] != '\n') ++pos;
                continue;
            }
            break;
        }
        if (pos >= text.size()) return false;
        const size_t b = pos;
        while (pos < text.size() && !isspace((unsigned char)text[pos]) && text[pos] != '#') ++pos;
        tok.assign(text, b, pos - b);
        return true;
    }
    bool fail(const std::string& m) {
        if (err.empty()) err = "line " + std::to_string(line) + ": " + m;
        return false;
    }
    bool expect(const char* key) {
        std::string t;
        if (!next(t)) return fail(std::string("expected '") + key + "', found end of file");
        if (t != key) return fail(std::string("expected '") + key + "', found '" + t + "'");
        return true;
    }
    bool number(double& v) {
        std::string t;
        if (!next(t)) return fail("expected a number, found end of file");
        char* end = nullptr;
        errno = 0;
        v = std::strtod(t.c_str(), &end);
        if (end == t.c_str() || *end != '\0' || errno == ERANGE) return fail("not a number: '" + t + "'");
        return true;
    }
    bool integer(int32_t& v, int lo, int hi) {
        double x;
        if (!number(x)) return false;
        if (x != (double)(int64_t)x || x < lo || x > hi) return fail("integer out of range");
        v = (int32_t)x;
        return true;
    }
    bool keyed_int(const char* key, int32_t& v, int lo, int hi) { return expect(key) && integer(v, lo, hi); }
    bool array(const char* key, size_t n, std::vector<double>& out) {
        if (!expect(key)) return false;
        out.resize(n);
        for (size_t k = 0; k < n; ++k)
            if (!number(out[k])) return false;
        return true;
    }
};

bool write_array(FILE* f, const char* key, const double* a, size_t n) {
    if (std::fprintf(f, "%s\n", key) < 0) return false;
    for (size_t k = 0; k < n; ++k)
        if (std::fprintf(f, "%.17g%c", a[k], (k % 8 == 7 || k + 1 == n) ? '\n' : ' ') < 0) return false;
    return true;
}

}  // namespace

extern "C" int tnep_model_save(const tnep_model_desc* d, const char* path) {
    if (!d || !path) {
        set_create_error("NULL argument");
        return TNEP_E_INVALID;
    }
    if (d->kind != TNEP_KIND_DIPOLE && d->kind != TNEP_KIND_POLARIZABILITY && d->kind != TNEP_KIND_PES) {
        set_create_error("unknown model kind");
        return TNEP_E_MODEL;
    }
    if (d->n_species < 1 || d->n_species > 8 || d->n_hidden < 1 || d->n_max_radial < 0 || d->n_max_angular < 0 ||
        d->basis_radial < 0 || d->basis_angular < 0 || d->l_max < 1) {
        set_create_error("model sizes out of range");
        return TNEP_E_MODEL;
    }
    const int heads = d->kind == TNEP_KIND_POLARIZABILITY ? 2 : 1;
    if (!d->c_radial || !d->c_angular || !d->q_scaler) {
        set_create_error("missing parameter arrays");
        return TNEP_E_MODEL;
    }
    for (int h = 0; h < heads; ++h)
        if (!d->w0[h] || !d->b0[h] || !d->w1[h] || (d->per_species && !d->b1_species[h])) {
            set_create_error("missing network arrays");
            return TNEP_E_MODEL;
        }
    FILE* f = std::fopen(path, "w");
    if (!f) {
        set_create_error(std::string("cannot open '") + path + "' for writing: " + std::strerror(errno));
        return TNEP_E_INVALID;
    }
    const size_t T = d->n_species, H = d->n_hidden, D = descriptor_length(*d);
    const size_t NS = d->per_species ? T : 1;
    bool ok = std::fprintf(f,
                           "tnep_model 1\nkind %s\nn_species %d\nrc %.17g %.17g\nn_max %d %d\nbasis %d %d\n"
                           "l_max %d\nfour_body %d\nfive_body %d\nn_hidden %d\nper_species %d\n",
                           kind_name(d->kind), d->n_species, d->rc_radial, d->rc_angular, d->n_max_radial,
                           d->n_max_angular, d->basis_radial, d->basis_angular, d->l_max, d->four_body ? 1 : 0,
                           d->five_body ? 1 : 0, d->n_hidden, d->per_species ? 1 : 0) > 0;
    ok = ok && write_array(f, "c_radial", d->c_radial, T * T * (d->n_max_radial + 1) * (d->basis_radial + 1));
    ok = ok && write_array(f, "c_angular", d->c_angular, T * T * (d->n_max_angular + 1) * (d->basis_angular + 1));
    ok = ok && write_array(f, "q_scaler", d->q_scaler, D);
    for (int h = 0; h < heads && ok; ++h) {
        ok = std::fprintf(f, "head %d\n", h) > 0;
        ok = ok && write_array(f, "w0", d->w0[h], NS * H * D);
        ok = ok && write_array(f, "b0", d->b0[h], NS * H);
        ok = ok && write_array(f, "w1", d->w1[h], NS * H);
        ok = ok && write_array(f, "b1", d->per_species ? d->b1_species[h] : &d->b1[h], NS);
    }
    ok = ok && std::fprintf(f, "end\n") > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        set_create_error(std::string("write to '") + path + "' failed");
        return TNEP_E_INVALID;
    }
    return TNEP_OK;
}

extern "C" int tnep_model_load(tnep_ctx* ctx, const char* path, tnep_model** out) {
    if (!ctx || !path || !out) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return c->fail(TNEP_E_INVALID, "cannot open '%s': %s", path, std::strerror(errno));
    Reader r;
    char buf[1 << 16];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) r.text.append(buf, n);
    std::fclose(f);

    tnep_model_desc d;
    std::memset(&d, 0, sizeof(d));
    std::string kind;
    int32_t version = 0;
    std::vector<double> cr, ca, qs, w0[2], b0[2], w1[2], b1[2];
    bool ok = r.keyed_int("tnep_model", version, 1, 1) && r.expect("kind") &&
              (r.next(kind) || r.fail("expected a model kind, found end of file"));
    if (ok) {
        if (kind == "dipole") d.kind = TNEP_KIND_DIPOLE;
        else if (kind == "polarizability") d.kind = TNEP_KIND_POLARIZABILITY;
        else if (kind == "pes") d.kind = TNEP_KIND_PES;
        else ok = r.fail("unknown kind '" + kind + "'");
    }
    // size limits keep a malformed header from asking for large arrays; the
    // supported shapes are checked by tnep_model_create
    ok = ok && r.keyed_int("n_species", d.n_species, 1, 8) && r.expect("rc") && r.number(d.rc_radial) &&
         r.number(d.rc_angular) && r.expect("n_max") && r.integer(d.n_max_radial, 0, 31) &&
         r.integer(d.n_max_angular, 0, 31) && r.expect("basis") && r.integer(d.basis_radial, 0, 31) &&
         r.integer(d.basis_angular, 0, 31) && r.keyed_int("l_max", d.l_max, 1, 8) &&
         r.keyed_int("four_body", d.four_body, 0, 1) && r.keyed_int("five_body", d.five_body, 0, 1) &&
         r.keyed_int("n_hidden", d.n_hidden, 1, 128) && r.keyed_int("per_species", d.per_species, 0, 1);
    const size_t T = d.n_species, H = d.n_hidden;
    const size_t D = ok ? descriptor_length(d) : 0;
    const size_t NS = d.per_species ? T : 1;
    ok = ok && r.array("c_radial", T * T * (d.n_max_radial + 1) * (d.basis_radial + 1), cr) &&
         r.array("c_angular", T * T * (d.n_max_angular + 1) * (d.basis_angular + 1), ca) &&
         r.array("q_scaler", D, qs);
    const int heads = d.kind == TNEP_KIND_POLARIZABILITY ? 2 : 1;
    for (int h = 0; h < heads && ok; ++h) {
        int32_t hh = -1;
        ok = r.keyed_int("head", hh, 0, 1);
        if (ok && hh != h) ok = r.fail("heads must be listed in order");
        ok = ok && r.array("w0", NS * H * D, w0[h]) && r.array("b0", NS * H, b0[h]) &&
             r.array("w1", NS * H, w1[h]) && r.array("b1", NS, b1[h]);
    }
    ok = ok && r.expect("end");
    std::string extra;
    if (ok && r.next(extra)) ok = r.fail("unexpected '" + extra + "' after 'end'");
    if (!ok) return c->fail(TNEP_E_MODEL, "model file '%s': %s", path, r.err.c_str());

    d.c_radial = cr.data();
    d.c_angular = ca.data();
    d.q_scaler = qs.data();
    for (int h = 0; h < heads; ++h) {
        d.w0[h] = w0[h].data();
        d.b0[h] = b0[h].data();
        d.w1[h] = w1[h].data();
        if (d.per_species)
            d.b1_species[h] = b1[h].data();
        else
            d.b1[h] = b1[h][0];
    }
    return tnep_model_create(ctx, &d, out);
}

"""Model files (tnep_model_save / tnep_model_load).

CPU: the writer needs no GPU; the file is read back here with a plain
tokenizer and every value must equal the model's FP64 parameters exactly
(17 significant digits round-trip).  GPU: a loaded model gives bitwise the
results of the same model created from memory, and malformed files are
rejected with TNEP_E_MODEL and the line number.
"""
import numpy as np
import pytest

import synth


def _tokens(path):
    out = []
    for line in open(path):
        out += line.split("#")[0].split()
    return out


def _models():
    a, b = synth.model("water_pes"), synth.model_raw("water_pes")
    b.heads = [synth.Head(h.w0 * 1.1, h.b0, h.w1, h.b1 + 0.2) for h in b.heads]
    return {
        "dipole": synth.model("water_dipole"),
        "polarizability_5b": synth.model("water_polarizability_5b"),
        "pes_per_species": synth.per_species_model([a, b], [1, 0]),
        "perovskite": synth.model("perovskite_susceptibility"),
    }


@pytest.mark.parametrize("name", list(_models()))
def test_save_writes_every_parameter_exactly(tmp_path, name):
    from paper_2312_05233_amd import tnep

    m = _models()[name]
    path = tmp_path / "m.tnep"
    tnep.tnep_model_save(m, str(path))
    tok = _tokens(path)
    kinds = {1: "dipole", 2: "polarizability", 3: "pes"}
    head = ["tnep_model", "1", "kind", kinds[m.kind], "n_species", str(len(m.species))]
    assert tok[:6] == head
    it = iter(tok[6:])

    def key(k):
        assert next(it) == k

    def nums(n):
        return np.array([float(next(it)) for _ in range(n)])

    key("rc")
    assert list(nums(2)) == [m.rc_radial, m.rc_angular]
    for k, v in (("n_max", [m.n_max_radial, m.n_max_angular]), ("basis", [m.basis_radial, m.basis_angular])):
        key(k)
        assert list(nums(2)) == v
    for k, v in (("l_max", m.l_max), ("four_body", int(m.four_body)), ("five_body", int(m.five_body)),
                 ("n_hidden", m.n_hidden), ("per_species", int(m.per_species))):
        key(k)
        assert nums(1)[0] == v
    for k, arr in (("c_radial", m.c_radial), ("c_angular", m.c_angular), ("q_scaler", m.q_scaler)):
        key(k)
        a = np.ravel(arr)
        assert np.array_equal(nums(a.size), a)
    for h, hd in enumerate(m.heads):
        key("head")
        assert nums(1)[0] == h
        for k, arr in (("w0", hd.w0), ("b0", hd.b0), ("w1", hd.w1), ("b1", np.atleast_1d(hd.b1))):
            key(k)
            a = np.ravel(arr)
            assert np.array_equal(nums(a.size), a), (name, h, k)
    key("end")
    assert next(it, None) is None


def test_save_errors(tmp_path):
    from paper_2312_05233_amd import tnep

    m = synth.model("water_dipole")
    with pytest.raises(tnep.TnepError) as e:
        tnep.tnep_model_save(m, str(tmp_path / "missing_dir" / "m.tnep"))
    assert e.value.code == -1 and "cannot open" in str(e.value)


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(_models()))
def test_loaded_model_matches_created(gpu_lib, tmp_path, name):
    m = _models()[name]
    path = tmp_path / "m.tnep"
    gpu_lib.tnep_model_save(m, str(path))
    ctx = gpu_lib.Context(0)
    a, b = gpu_lib.Model(ctx, m), gpu_lib.Model.load(ctx, str(path))
    assert b.kind == m.kind
    fr = synth.perovskite(1, n_rep=4) if name == "perovskite" else synth.water_small(2, seed=71)
    if m.kind == synth.KIND_PES:
        for x, y in zip(gpu_lib.tnep_eval_pes(ctx, a, fr), gpu_lib.tnep_eval_pes(ctx, b, fr)):
            assert np.array_equal(x, y)
    else:
        f = gpu_lib.tnep_eval_dipole if m.kind == synth.KIND_DIPOLE else gpu_lib.tnep_eval_polarizability
        assert np.array_equal(f(ctx, a, fr), f(ctx, b, fr))
    ctx.close()


@pytest.mark.gpu
def test_malformed_files_are_rejected(gpu_lib, tmp_path):
    m = synth.model("water_dipole")
    good = tmp_path / "good.tnep"
    gpu_lib.tnep_model_save(m, str(good))
    text = good.read_text()
    lines = text.splitlines(keepends=True)
    cases = {
        "truncated": "".join(lines[: len(lines) // 2]),
        "bad_keyword": text.replace("basis 8 8", "basis_size 8 8"),
        "bad_number": text.replace("rc 6 4", "rc 6 four"),
        "unsupported_shape": text.replace("n_max 4 4", "n_max 3 4"),
        "trailing": text + "extra\n",
        "wrong_kind": text.replace("kind dipole", "kind quadrupole"),
    }
    ctx = gpu_lib.Context(0)
    for label, body in cases.items():
        p = tmp_path / (label + ".tnep")
        p.write_text(body)
        with pytest.raises(gpu_lib.TnepError) as e:
            gpu_lib.Model.load(ctx, str(p))
        assert e.value.code == -7, label
        if label != "unsupported_shape":
            assert "line" in str(e.value), label
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.Model.load(ctx, str(tmp_path / "absent.tnep"))
    assert e.value.code == -1
    # comments are allowed anywhere
    p = tmp_path / "commented.tnep"
    p.write_text("# a water dipole model\n" + text.replace("n_hidden 30", "n_hidden 30  # H"))
    fr = synth.water_small(1, seed=72)
    assert np.array_equal(gpu_lib.tnep_eval_dipole(ctx, gpu_lib.Model.load(ctx, str(p)), fr),
                          gpu_lib.tnep_eval_dipole(ctx, gpu_lib.Model(ctx, m), fr))
    ctx.close()

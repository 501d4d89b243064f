"""The pins catch planted mistakes.  Each case copies oracle/oracle.c, plants
one plausible error by a textual substitution (a dropped or wrong term, a
wrong sign, an off-by-one), builds the copy with gcc into a temporary folder,
points the oracle at it, and checks that a pin rejects it: the Jordan-Wigner
entry pin (every entry of H against an independent Fock-space construction,
all sectors) for mistakes in H, the finite-difference pin for mistakes in the
parameter bilinear forms.  The oracle's own source and library are not
touched."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_pins import _jordan_wigner_H, test_hellmann_feynman_vs_finite_differences

MUTATIONS = [
    ("sign counts an endpoint", "for (int k = p + 1; k < q; ++k)", "for (int k = p; k < q; ++k)"),
    ("fermionic sign dropped", "*sign = (between & 1) ? -1.0 : 1.0;", "*sign = 1.0;"),
    ("U on n_up + n_dn", "d += m->U[i] * (double)(nu * nd);", "d += m->U[i] * (double)(nu + nd);"),
    ("eps of the down spin dropped", "if (m->eps) d += m->eps[i] * (double)(nu + nd);",
     "if (m->eps) d += m->eps[i] * (double)(nu);"),
    ("hopping sign flipped", "e[n].val = -m->t[b] * sg;", "e[n].val = m->t[b] * sg;"),
    ("spins mixed in a hop", "int q = m->bj[b] + s * m->M;", "int q = m->bj[b] + (1 - s) * m->M;"),
]

# mistakes in the parameter bilinear forms only (H itself intact): caught by
# the finite-difference pin of the Hellmann-Feynman derivatives
BILINEAR_MUTATIONS = [
    ("dU on n_up + n_dn", "a[nb + i] += (double)(nu * nd) * gx;", "a[nb + i] += (double)(nu + nd) * gx;"),
    ("bond form sign flipped", "a[b] += -sg * g[r] * x[c];", "a[b] += sg * g[r] * x[c];"),
    ("deps without the down spin", "a[nb + M + i] += (double)(nu + nd) * gx;",
     "a[nb + M + i] += (double)(nu) * gx;"),
]


def _pin_holds(model):
    """The entry pin of test_jordan_wigner_entries on one lattice, all sectors."""
    Hf = _jordan_wigner_H(model).tocsr()
    M = model.n_sites
    for n_up in range(M + 1):
        for n_dn in range(M + 1):
            sec = oracle.Sector(model.with_params(n_up=n_up, n_dn=n_dn))
            keys = sec.keys.astype(np.int64)
            if not np.allclose(sec.dense(), Hf[keys][:, keys].toarray(), rtol=0, atol=1e-14):
                return False
    return True


def _model():
    base = W.random_graph(4, 5, seed=2, site_U=True)
    return base.with_params(eps=[0.3, -0.7, 0.11, 0.5])


def test_unmutated_oracle_passes_the_pin():
    assert _pin_holds(_model())


def _use_mutant(tmp_path, monkeypatch, old, new):
    """Build oracle.c with `old` replaced by `new` and make the oracle load it."""
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, old
    mut = tmp_path / "oracle_mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(mut),
                           "-lm"])
    monkeypatch.setattr(oracle, "_SRC", str(mut))
    monkeypatch.setattr(oracle, "_LIB", str(so))
    monkeypatch.setattr(oracle, "_lib", None)


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_rejects_planted_mistake(tmp_path, monkeypatch, name, old, new):
    _use_mutant(tmp_path, monkeypatch, old, new)
    try:
        held = _pin_holds(_model())
    except Exception:  # a mutant may also fail loudly (e.g. a target state outside the sector)
        held = False
    assert not held, f"the pin did not catch: {name}"


@pytest.mark.parametrize("name,old,new", BILINEAR_MUTATIONS, ids=[m[0] for m in BILINEAR_MUTATIONS])
def test_finite_difference_pin_rejects_planted_mistake(tmp_path, monkeypatch, name, old, new):
    _use_mutant(tmp_path, monkeypatch, old, new)
    with pytest.raises(AssertionError):
        test_hellmann_feynman_vs_finite_differences()


# mistakes in the Green's-function oracle's fermion operator (Python): caught by
# its pin against the Jordan-Wigner Fock-space operators
OPERATOR_MUTATIONS = [
    ("sign counts the mode itself", "keys[cols] & (bit - np.uint64(1))",
     "keys[cols] & ((bit << np.uint64(1)) - np.uint64(1))"),
    ("sign counts the modes above", "keys[cols] & (bit - np.uint64(1))",
     "keys[cols] & ~((bit << np.uint64(1)) - np.uint64(1))"),
    ("create and annihilate swapped", "take = ~occupied if create else occupied",
     "take = occupied if create else ~occupied"),
]


@pytest.mark.parametrize("name,old,new", OPERATOR_MUTATIONS, ids=[m[0] for m in OPERATOR_MUTATIONS])
def test_operator_pin_rejects_planted_mistake(monkeypatch, name, old, new):
    import inspect
    import textwrap
    import oracle.greens as og
    from test_oracle_greens import test_fermion_operator_matches_jordan_wigner
    src = textwrap.dedent(inspect.getsource(og.fermion_operator))
    assert src.count(old) == 1, name
    ns = dict(vars(og))
    exec(compile(src.replace(old, new), og.__file__, "exec"), ns)
    monkeypatch.setattr(og, "fermion_operator", ns["fermion_operator"])
    with pytest.raises(AssertionError):
        test_fermion_operator_matches_jordan_wigner(12, 4)


def _mutate_function(module, fname, old, new, monkeypatch):
    """Replace module.fname by a copy of its source with `old` replaced by `new`."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(getattr(module, fname)))
    assert src.count(old) == 1, (fname, old)
    ns = dict(vars(module))
    exec(compile(src.replace(old, new), module.__file__, "exec"), ns)
    monkeypatch.setattr(module, fname, ns[fname])


def _fails(*checks):
    """True when any of the pin functions raises an AssertionError."""
    for check in checks:
        try:
            check()
        except AssertionError:
            return True
    return False


# mistakes in the translation oracle's signs: caught by the Table VI fixture and
# T^2 |0101> = -|0101> (one-spin cycles) or by [H, T] = 0 and the group-projector
# construction (two-spin translation operator)
def test_translation_pins_reject_planted_sign_mistakes(monkeypatch):
    import oracle.translation as ot
    import test_oracle_translation as tt
    with monkeypatch.context() as mp:
        _mutate_function(ot, "gsign", "(k * (N - k)) % 2", "(k * N) % 2", mp)
        assert _fails(tt.test_table6_spin_table, tt.test_t_squared_on_0101)
    projector = [lambda i=i: tt.test_k0_block_against_group_projector(i) for i in range(7)]
    with monkeypatch.context() as mp:
        _mutate_function(ot, "_key_rotate", "np.where((k * (N - k)) % 2 == 1, -1.0, 1.0)",
                         "np.where(k % 2 == 1, -1.0, 1.0)", mp)
        assert _fails(*projector)
    with monkeypatch.context() as mp:
        _mutate_function(ot, "_key_rotate", "sgn(up, n_up) * sgn(dn, n_dn)", "sgn(up, n_up)", mp)
        assert _fails(*projector)
    # and the unmutated oracle passes them all
    tt.test_table6_spin_table()
    tt.test_t_squared_on_0101()
    for check in projector:
        check()


def test_solver_and_generator_pins_reject_planted_mistakes(tmp_path, monkeypatch):
    """The oracle's Lanczos without the beta term fails the LAPACK pin; a
    continued fraction with b instead of b^2 fails the closed forms; a SplitMix64
    with a wrong shift fails the reference outputs."""
    import oracle.greens as og
    import test_oracle_greens as tg
    import test_oracle_pins as tp
    with monkeypatch.context() as mp:
        _mutate_function(oracle, "lanczos", "w = matvec(v) - beta * v_prev\n        a = float(",
                         "w = matvec(v)\n        a = float(", mp)
        assert _fails(lambda: tp.test_lanczos_matches_dense(21), lambda: tp.test_lanczos_matches_dense(22))
    with monkeypatch.context() as mp:
        _mutate_function(og, "continued_fraction", "betas[j] ** 2 / d", "betas[j] / d", mp)
        assert _fails(tg.test_continued_fraction_closed_forms, tg.test_continued_fraction_matches_lehmann)
    with monkeypatch.context() as mp:
        _use_mutant(tmp_path, mp, "z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;",
                    "z = (z ^ (z >> 28)) * 0x94D049BB133111EBull;")
        assert _fails(tp.test_splitmix64_reference_outputs)

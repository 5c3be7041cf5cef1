"""Host code of the library on the CPU (no GPU):

* fscc_heff_eig (the diagonalisation of H_eff, step V of the flowchart) on
  matrices whose spectra are known: diagonal and triangular matrices (exact),
  similarity transforms X diag(d) X^-1 of chosen eigenvalues, companion
  matrices of polynomials with chosen roots, Hermitian matrices (real spectra,
  cross-checked against LAPACK's Hermitian solver), a rotation with +-i,
  random matrices against LAPACK's general solver; ordering and error codes;
* the divergence rule of the amplitude update (csrc/diverge.hpp, compiled
  with g++): geometric growth is answered by one DIIS reset and then by
  giving up, noise at the rounding floor and ordinary DIIS fluctuations are
  not, non-finite steps give up at once.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2004_03682_amd", "csrc")


def _eig(a):
    import paper_2004_03682_amd as F
    return F.heff_eig(a)


def _sorted(w):
    w = np.asarray(w, np.complex128)
    return w[np.lexsort((w.imag, w.real))]


def _match(w, ref):
    """Largest distance from an eigenvalue to the nearest reference value, after
    checking that the two lists have the same length and w is sorted by real part
    (values whose real parts tie to rounding may come in either order)."""
    assert w.size == ref.size and np.all(np.diff(w.real) >= -1e-12 * max(1.0, np.abs(w).max()))
    return max(np.abs(ref - x).min() for x in w) if w.size else 0.0


def test_diagonal_and_triangular_are_exact():
    rng = np.random.default_rng(1)
    d = rng.normal(size=9) + 1j * rng.normal(size=9)
    assert np.array_equal(_eig(np.diag(d)), _sorted(d))
    u = np.triu(rng.normal(size=(9, 9)) + 1j * rng.normal(size=(9, 9)), 1) + np.diag(d)
    assert np.array_equal(_eig(u), _sorted(d))
    assert np.array_equal(_eig(np.array([[1.0, 1.0], [0.0, 1.0]])), np.array([1.0, 1.0]))
    assert _eig(np.zeros((0, 0))).size == 0
    assert np.array_equal(_eig(np.array([[2.5 - 1j]])), np.array([2.5 - 1j]))


@pytest.mark.parametrize("n,seed", [(2, 3), (6, 4), (15, 5), (40, 6)])
def test_similarity_transform_of_known_eigenvalues(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=n) + 1j * rng.normal(size=n)
    X = np.eye(n) + 0.3 * (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
    a = X @ np.diag(d) @ np.linalg.inv(X)
    w = _eig(a)
    # eigenvalue error ~ cond(X) * eps * |A|
    tol = 1e-13 * np.linalg.cond(X) * np.abs(a).max() * n
    assert _match(w, d) <= tol


def test_companion_matrix_roots():
    roots = np.array([1.0, -2.0, 0.5 + 1.5j, 0.5 - 1.5j, 3j, -1.25 + 0.25j])
    c = np.poly(roots)                      # monic coefficients, highest first
    n = roots.size
    comp = np.zeros((n, n), np.complex128)
    comp[0, :] = -c[1:]
    comp[1:, :-1] = np.eye(n - 1)
    assert _match(_eig(comp), roots) <= 1e-11


@pytest.mark.parametrize("n,seed", [(6, 7), (15, 8), (64, 9)])
def test_hermitian_spectrum_is_real_and_matches_lapack(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    h = x + x.conj().T
    w = _eig(h)
    scale = np.abs(h).max() * n
    assert np.abs(w.imag).max() <= 1e-13 * scale
    assert np.abs(w.real - np.linalg.eigvalsh(h)).max() <= 1e-13 * scale


def test_rotation_has_eigenvalues_plus_minus_i():
    w = _eig(np.array([[0.0, 1.0], [-1.0, 0.0]]))
    assert np.abs(w - np.array([-1j, 1j])).max() <= 1e-15


@pytest.mark.parametrize("n,seed", [(6, 10), (15, 11), (100, 12)])
def test_random_matrices_match_lapack(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    w = _eig(a)
    assert _match(w, np.linalg.eigvals(a)) <= 1e-11 * np.abs(a).max() * n


def test_rejects_bad_input():
    import paper_2004_03682_amd as F
    with pytest.raises(F.FsccError):
        _eig(np.array([[1.0, np.nan], [0.0, 1.0]]))
    with pytest.raises(ValueError):
        _eig(np.zeros((2, 3)))
    assert F.lib().fscc_heff_eig(-1, None, None) == -1
    assert F.lib().fscc_heff_eig(3, None, None) == -1


@pytest.fixture(scope="module")
def watch(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("host") / "libdiverge.so")
    subprocess.run([gxx, "-O1", "-std=c++17", "-shared", "-fPIC", "-I" + CSRC, "-o", out,
                    os.path.join(HERE, "host", "diverge_check.cpp")], check=True)
    lib = ctypes.CDLL(out)

    def run(steps):
        steps = np.ascontiguousarray(steps, dtype=np.float64)
        act = np.zeros(steps.size, dtype=np.int32)
        lib.diverge_actions(steps.ctypes.data_as(ctypes.c_void_p), int(steps.size), act.ctypes.data_as(ctypes.c_void_p))
        return act

    g, f = ctypes.c_double(), ctypes.c_double()
    lib.diverge_constants(ctypes.byref(g), ctypes.byref(f))
    return run, g.value, f.value


CONTINUE, RESET, GIVE_UP = 0, 1, 2


def test_converging_and_fluctuating_runs_continue(watch):
    run, growth, floor = watch
    # a DIIS-like run: up-and-down steps that decrease overall, then rounding noise
    steps = [1.5e-2, 4.0e-2, 8e-3, 1.1e-2, 1.3e-2, 2e-3, 5e-3, 1e-4, 3e-4, 1e-6, 1e-8, 1e-10, 1e-12,
             3e-14, 1e-16, 2e-13, 1e-15, 5e-14]
    assert np.all(run(steps) == CONTINUE)
    # growth just below the factor is tolerated
    assert np.all(run([1e-2, 0.99 * growth * 1e-2]) == CONTINUE)


def test_geometric_growth_resets_then_gives_up(watch):
    run, growth, floor = watch
    steps = 0.05 * 1.5 ** np.arange(60)
    act = run(steps)
    k_reset = int(np.argmax(act == RESET))
    assert act[k_reset] == RESET and np.all(act[:k_reset] == CONTINUE)
    assert steps[k_reset] > growth * steps[0] and steps[k_reset - 1] <= growth * steps[0]
    k_stop = int(np.argmax(act == GIVE_UP))
    assert k_stop > k_reset and np.all(act[k_reset + 1:k_stop] == CONTINUE)
    assert steps[k_stop] > growth * steps[k_reset] and steps[k_stop - 1] <= growth * steps[k_reset]


def test_floor_keeps_rounding_noise_from_counting_as_growth(watch):
    run, growth, floor = watch
    # from 1e-16 a jump to just below growth * floor is noise, above it is growth
    assert np.all(run([1e-16, 0.9 * growth * floor]) == CONTINUE)
    assert list(run([1e-16, 1.1 * growth * floor])) == [CONTINUE, RESET]


def test_non_finite_steps_give_up_at_once(watch):
    run, growth, floor = watch
    assert list(run([1e-2, np.nan])) == [CONTINUE, GIVE_UP]
    assert list(run([np.inf])) == [GIVE_UP]

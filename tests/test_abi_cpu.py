"""CPU-only checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments with reference-BLAS numbering before
touching a GPU. No compute call is made here."""
import os
import re

import pytest

import paper_2603_29975_amd as oz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h") or fn == "ozaki_blas.h":   # the interposer: test_blas_cpu.py
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ozaki2?_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = oz.library()
    names = _declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    for name in _declared_functions():
        assert hasattr(oz, name), name


@pytest.mark.parametrize("fn", ["ozaki_dgemm", "ozaki_zgemm", "ozaki2_dgemm", "ozaki2_zgemm"])
def test_gemm_argument_errors(fn):
    f = getattr(oz, fn)
    ok = dict(transa="N", transb="N", m=4, n=5, k=6, alpha=1.0, A=0, lda=4, B=0, ldb=6, beta=0.0,
              C=0, ldc=4, slices=7)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return f(a["transa"], a["transb"], a["m"], a["n"], a["k"], a["alpha"], a["A"], a["lda"],
                 a["B"], a["ldb"], a["beta"], a["C"], a["ldc"], a["slices"])

    assert call(transa="X") == -1
    assert call(transb="Q") == -2
    assert call(m=-1) == -3
    assert call(n=-1) == -4
    assert call(k=-1) == -5
    assert call(lda=3) == -8
    assert call(transa="T", lda=5) == -8          # rows of A as stored = k = 6
    assert call(ldb=5) == -10
    assert call(transb="C", ldb=4) == -10         # rows of B as stored = n = 5
    assert call(ldc=3) == -13
    assert call(slices=0) == -14
    assert call(slices=21 if fn.startswith("ozaki2") else 13) == -14
    if fn.startswith("ozaki2"):
        assert call(slices=1) == -14
    assert call(C=0) == -12                       # null C with work to do
    assert call(m=0) == 0 and call(n=0) == 0      # quick returns, nothing launched
    assert call(A=0, C=1 << 40) == -7             # null A with alpha != 0 and k > 0
    assert call(transa="n", transb="c", A=1 << 40, B=0, C=1 << 40, lda=4) == -9


@pytest.mark.parametrize("fn", ["ozaki_native_dgemm", "ozaki_native_zgemm"])
def test_native_argument_errors(fn):
    f = getattr(oz, fn)
    assert f("X", "N", 1, 1, 1, 1.0, 0, 1, 0, 1, 0.0, 0, 1) == -1
    assert f("N", "N", 4, 1, 1, 1.0, 0, 3, 0, 1, 0.0, 0, 4) == -8
    assert f("N", "N", 4, 2, 3, 1.0, 0, 4, 0, 2, 0.0, 0, 4) == -10
    assert f("N", "N", 4, 2, 3, 1.0, 0, 4, 0, 3, 0.0, 0, 3) == -13
    assert f("N", "N", 0, 2, 3, 1.0, 0, 4, 0, 3, 0.0, 0, 4) == 0


def test_debug_hook_argument_errors():
    assert oz.ozaki_debug_exponents("q", "A", "N", 1, 1, 0, 1, 0, 0) == -1
    assert oz.ozaki_debug_exponents("d", "x", "N", 1, 1, 0, 1, 0, 0) == -2
    assert oz.ozaki_debug_exponents("d", "A", "y", 1, 1, 0, 1, 0, 0) == -3
    assert oz.ozaki_debug_exponents("d", "A", "N", -1, 1, 0, 1, 0, 0) == -4
    assert oz.ozaki_debug_exponents("d", "A", "N", 3, 1, 0, 2, 0, 0) == -7
    assert oz.ozaki_debug_split("z", "B", "N", 2, 3, 1 << 40, 3, 0, 0) == -8
    assert oz.ozaki_debug_diagonals("x", "N", "N", 1, 1, 1, 0, 1, 0, 1, 3, 0) == -100
    assert oz.ozaki_debug_diagonals("d", "N", "N", 1, 1, 1, 0, 1, 0, 1, 13, 0) == -14


def test_status_strings_and_workspace_sizes():
    assert oz.ozaki_status_string(0) == "success"
    assert oz.ozaki_status_string(-4) == "invalid argument"
    assert oz.ozaki_status_string(2) != oz.ozaki_status_string(1)
    assert oz.ozaki_workspace_bytes("q", 1, 1, 1, 7) == 0
    assert oz.ozaki_workspace_bytes("d", 1, 1, 1, 13) == 0
    small = oz.ozaki_workspace_bytes("d", 256, 256, 256, 7)
    big = oz.ozaki_workspace_bytes("z", 256, 256, 256, 7)
    assert 0 < small < big
    # packed slices dominate: s bytes per padded real entry of A' and B'
    assert oz.ozaki_workspace_bytes("d", 256, 256, 256, 8) > small
    assert small >= 7 * (256 * 256 + 256 * 256)


def test_batched_argument_errors():
    z = [0]
    ok = dict(transa=["N"], transb=["N"], m=[4], n=[5], k=[6], alpha=[1.0], A=[1 << 40], lda=[4],
              B=[1 << 40], ldb=[6], beta=[0.0], C=[1 << 40], ldc=[4], batch=1, slices=[7])

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return oz.ozaki_zgemm_batched(a["transa"], a["transb"], a["m"], a["n"], a["k"], a["alpha"],
                                      a["A"], a["lda"], a["B"], a["ldb"], a["beta"], a["C"],
                                      a["ldc"], a["batch"], a["slices"])

    assert call(batch=-1) == -14
    assert call(batch=0) == 0
    assert call(transa=["x"]) == -1
    assert call(m=[-2]) == -3
    assert call(lda=[2]) == -8
    assert call(ldc=[1]) == -13
    assert call(slices=[0]) == -15
    assert call(slices=[13]) == -15
    assert call(C=[0]) == -12
    assert call(A=[0]) == -7
    assert call(slices=None) == 6          # OZAKI_ERR_NO_SELECTOR: automatic mode needs a selector
    del z


def test_probe_argument_errors():
    f = oz.ozaki_probe
    assert f("x", "N", "N", 2, 2, 2, 1, 2, 1, 2, 1, 2, 1, 0, 1) == -1
    assert f("d", "Q", "N", 2, 2, 2, 1, 2, 1, 2, 1, 2, 1, 0, 1) == -2
    assert f("d", "N", "Q", 2, 2, 2, 1, 2, 1, 2, 1, 2, 1, 0, 1) == -3
    assert f("d", "N", "N", -1, 2, 2, 1, 2, 1, 2, 1, 2, 1, 0, 1) == -4
    assert f("d", "N", "N", 2, 2, 2, 1, 1, 1, 2, 1, 2, 1, 0, 1) == -8
    assert f("d", "N", "N", 2, 2, 2, 1, 2, 1, 1, 1, 2, 1, 0, 1) == -10
    assert f("d", "N", "N", 2, 2, 2, 1, 2, 1, 2, 1, 1, 1, 0, 1) == -12
    assert f("d", "N", "N", 2, 2, 2, 1, 2, 1, 2, 1, 2, 5, 0, 1) == -13
    assert f("d", "N", "N", 2, 2, 2, 1, 2, 1, 2, 1, 2, 1, 0, 0) == -15
    assert f("d", "N", "N", 0, 2, 2, 1, 2, 1, 2, 1, 2, 1, 0, 0) == 0


def test_tuning_table_host_logic():
    # The tuning table is host state: set / get / clear work without a GPU.
    assert oz.ozaki_tune_clear() == 0
    nid = oz.ozaki_tune_configs()
    assert nid == 28                       # 7 tile configurations x 4 tile orders
    assert oz.ozaki_tune_get("z", 2048, 2048, 2048, 7) == 0          # default id
    assert oz.ozaki_tune_set("z", 2048, 2048, 2048, 7, nid - 1) == 0
    assert oz.ozaki_tune_get("z", 2048, 2048, 2048, 7) == nid - 1
    # same buckets (ceil log2 of m, n', 32-deep blocks of k'): 1500 -> 11, 2n = 3000 -> 12
    assert oz.ozaki_tune_get("z", 1500, 1500, 1500, 7) == nid - 1
    assert oz.ozaki_tune_get("z", 2049, 2048, 2048, 7) == 0          # next m bucket
    assert oz.ozaki_tune_get("z", 2048, 2048, 2048, 6) == 0          # other slice count
    assert oz.ozaki_tune_get("d", 2048, 4096, 4096, 7) == 0          # real data: own entries
    assert oz.ozaki_tune_set("z", 2048, 2048, 2048, 7, -1) == 0      # remove
    assert oz.ozaki_tune_get("z", 2048, 2048, 2048, 7) == 0
    assert oz.ozaki_tune_set("d", 64, 64, 64, 3, 1) == 0
    assert oz.ozaki_tune_clear() == 0
    assert oz.ozaki_tune_get("d", 64, 64, 64, 3) == 0
    # argument errors
    assert oz.ozaki_tune_set("q", 1, 1, 1, 7, 0) == -1
    assert oz.ozaki_tune_set("d", 0, 1, 1, 7, 0) == -2
    assert oz.ozaki_tune_set("d", 1, 0, 1, 7, 0) == -3
    assert oz.ozaki_tune_set("d", 1, 1, 0, 7, 0) == -4
    assert oz.ozaki_tune_set("d", 1, 1, 1, 13, 0) == -5
    assert oz.ozaki_tune_set("d", 1, 1, 1, 7, nid) == -6
    assert oz.ozaki_tune_get("z", 1, 1, 1, 0) == -5
    rc, best, _ = oz.ozaki_autotune("d", 8, 8, 8, 7, reps=0)
    assert rc == -6 and best == -1
    assert oz.ozaki_autotune("x", 8, 8, 8, 7)[0] == -1
    assert oz.ozaki_tune_save(None) == -1 and oz.ozaki_tune_load(None) == -1


def test_ozaki2_host_logic_matches_the_oracle():
    # moduli and the bit budget beta: the library's host tables against the
    # oracle's definitions (reading Q1/Q2), without device work
    from oracle import ozaki2
    for n in range(oz.MODULI_MIN, oz.MODULI_MAX + 1):
        rc, mods = oz.ozaki2_moduli(n)
        assert rc == 0 and mods == ozaki2.moduli(n)
        for kp in (1, 2, 3, 64, 100, 4096, 4097, 65536, 131072):
            try:
                want = ozaki2.beta_bits(n, kp)
            except ValueError:
                want = 0
            assert oz.ozaki2_beta_bits(n, kp) == want, (n, kp)
    assert oz.ozaki2_moduli(1)[0] == -1 and oz.ozaki2_moduli(21)[0] == -1
    assert oz.ozaki2_beta_bits(14, 0) == -2 and oz.ozaki2_beta_bits(14, oz.K2_MAX + 1) == -2


def test_ozaki2_size_limits_and_workspace():
    big = 1 << 40
    # K' beyond exact INT32 modular sums: k for real, 2k for complex
    assert oz.ozaki2_dgemm("N", "N", 4, 4, oz.K2_MAX + 1, 1.0, big, 4, big, oz.K2_MAX + 1, 0.0,
                           big, 4, 14) == -5
    assert oz.ozaki2_zgemm("N", "N", 4, 4, oz.K2_MAX // 2 + 1, 1.0, big, 4, big,
                           oz.K2_MAX // 2 + 1, 0.0, big, 4, 14) == -5
    # two moduli leave no bits for K' = 2^13 (beta < 1)
    assert oz.ozaki2_dgemm("N", "N", 4, 4, 8192, 1.0, big, 4, big, 8192, 0.0, big, 4, 2) == -14
    assert oz.ozaki2_workspace_bytes("d", 4, 4, 8192, 2) == 0
    assert oz.ozaki2_workspace_bytes("z", 4, 4, oz.K2_MAX, 14) == 0
    w14 = oz.ozaki2_workspace_bytes("z", 256, 256, 256, 14)
    # residues of A' (256 x 512) and B' (512 x 512) per modulus, and nothing for the
    # INT32 products (they stay in registers)
    assert 14 * (256 * 512 + 512 * 512) <= w14 < 14 * (256 * 512 + 512 * 512) + 8192
    assert oz.ozaki2_workspace_bytes("z", 256, 256, 256, 16) > w14
    assert oz.ozaki2_workspace_bytes("q", 4, 4, 4, 14) == 0


def test_lu_argument_errors():
    big = 1 << 40
    assert oz.ozaki_zgetrf(-1, big, 4, big, 64, 6) == -1
    assert oz.ozaki_zgetrf(4, 0, 4, big, 64, 6) == -2
    assert oz.ozaki_zgetrf(4, big, 3, big, 64, 6) == -3
    assert oz.ozaki_zgetrf(4, big, 4, 0, 64, 6) == -4
    assert oz.ozaki_zgetrf(4, big, 4, big, 0, 6) == -5
    assert oz.ozaki_zgetrf(4, big, 4, big, 64, -1) == -6
    assert oz.ozaki_zgetrf(0, 0, 1, 0, 64, 6) == 0
    assert oz.ozaki_zgetri(4, big, 4, big, 0, 4, 64, 6) == -7
    assert oz.ozaki_zgetri(4, big, 4, big, big, 3, 64, 6) == -8

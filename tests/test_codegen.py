"""The per-network code generator, on the CPU: the generated source's
structure (the network's stoichiometry, coefficients and sparsity as
constants, sums in ascending reaction order), its LU fill pattern against a
symbolic elimination written here, its compilation for gfx950 without a GPU
(hiprtc) and the code-object cache, and the cases it refuses."""
import os
import re

import numpy as np
import pytest

from paper_2312_02836_amd import synth


@pytest.fixture(scope="module")
def B():
    from paper_2312_02836_amd import burn
    return burn


def _patterns(spec):
    """Jacobian pattern of f = (dY/dt, dT/dt) and the LU fill of I - cJ with
    diagonal pivots, by plain symbolic elimination over sets."""
    N, n = spec.n_species, spec.n
    J = [set() for _ in range(n)]
    for r in range(spec.n_reactions):
        rs = {int(x) for x in spec.reactants[r] if x >= 0}
        ps = [int(x) for x in spec.products[r] if x >= 0]
        for i in range(N):
            nu = ps.count(i) - [int(x) for x in spec.reactants[r]].count(i)
            if nu:
                J[i] |= rs | {N}
        J[N] |= rs | {N}
    F = [set(J[i]) | {i} for i in range(n)]
    for K in range(n):
        for i in range(K + 1, n):
            if K in F[i]:
                F[i] |= {j for j in F[K] if j > K}
    return J, F


def _consts(src, name):
    m = re.search(name + r"\[[^\]]*\] = \{([^}]*)\}", src)
    return [int(x.strip().rstrip("ull"), 16) for x in m.group(1).split(",")]


@pytest.mark.parametrize("cfg_i,which", [(2, 0), (4, 0), (1, 0)])
def test_fill_pattern_matches_symbolic_elimination(B, cfg_i, which):
    spec = synth.config(cfg_i, n_cells=4).networks[which]
    src = B.codegen_source(spec)
    _, F = _patterns(spec)
    fpat = _consts(src, "fpat")
    assert len(fpat) == spec.n
    for i in range(spec.n):
        assert fpat[i] == sum(1 << j for j in F[i]), i


def test_source_holds_the_network(B):
    spec = synth.config(2, n_cells=4).networks[0]
    src = B.codegen_source(spec, 2)
    assert f"N = {spec.n_species}, R = {spec.n_reactions}" in src
    assert "2 lane(s) per cell" in src
    # every rate coefficient appears as an exact hexadecimal constant
    consts = {float.fromhex(m) for m in re.findall(r"-?0x[0-9a-f.]+p[+-]\d+", src)}
    for r in range(spec.n_reactions):
        for c in spec.coef[r]:
            assert float(c) in consts
    # the right-hand side sums run in ascending reaction order: for every
    # species, the reactions it takes part in appear in order of r
    rhs = src[src.index("static void rhs("):src.index("static constexpr int NE")]
    for i in range(spec.n_species):
        rs = [int(m.group(1)) for m in re.finditer(rf"f{i} = f{i} \+ [^;]*?r(\d+)\b", rhs)]
        nus = [r for r in range(spec.n_reactions)
               if list(spec.products[r]).count(i) != list(spec.reactants[r]).count(i)]
        assert rs == nus, (i, rs, nus)
    assert "#pragma clang fp contract(off)" in src


def test_lane_choice_and_refusals(B):
    from paper_2312_02836_amd import _lib
    small = synth.reversible_pair(3.0, 0.5)
    assert "1 lane(s) per cell" in B.codegen_source(small)
    assert "2 lane(s) per cell" in B.codegen_source(small, 2)
    big = synth.config(4, n_cells=4).networks[1]  # 21/60: 22 components
    with pytest.raises(_lib.BurnError):
        B.codegen_source(big)
    scr = synth.screened(synth.config(2, n_cells=4).networks[0])
    with pytest.raises(_lib.BurnError):
        B.codegen_source(scr)
    with pytest.raises(_lib.BurnError):
        B.codegen_source(synth.config(2, n_cells=4).networks[0], 1)  # 14 components, one lane


def test_prebuild_compiles_and_caches(B, tmp_path):
    """hiprtc compiles the generated source for gfx950 without a GPU; the
    code object lands in the cache once and is found there again."""
    spec = synth.chain_network([3.0, 0.7, 0.05], q=[1.0, 2.0, 0.5])
    d = str(tmp_path / "cache")
    B.codegen_prebuild(spec, 0, d)
    files = os.listdir(d)
    assert len(files) == 1 and files[0].startswith("bng_") and files[0].endswith(".co")
    blob = open(os.path.join(d, files[0]), "rb").read()
    assert blob[:4] == b"\x7fELF"
    mtime = os.path.getmtime(os.path.join(d, files[0]))
    B.codegen_prebuild(spec, 0, d)
    assert os.listdir(d) == files and os.path.getmtime(os.path.join(d, files[0])) == mtime
    # another network: another key
    B.codegen_prebuild(synth.reversible_pair(3.0, 0.5), 0, d)
    assert len(os.listdir(d)) == 2


def test_prebuild_of_the_benchmark_network(B, tmp_path):
    spec = synth.config(2, n_cells=4).networks[0]
    B.codegen_prebuild(spec, 0, str(tmp_path))
    (f,) = os.listdir(tmp_path)
    assert os.path.getsize(tmp_path / f) > 10000

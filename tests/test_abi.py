"""The C-ABI library loads on the CPU and exports every entry point include/tvmc.h declares
(no compute calls: there may be no GPU here)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvmc.h")
LIB = os.path.join(ROOT, "paper_2506_23928_amd", "libtvmc.so")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:tvmc_status|const char \*)\s*(tvmc_\w+)\s*\(", src, re.M)))


def test_header_declares_the_stage_calls():
    names = _declared()
    for n in ("tvmc_init", "tvmc_sample", "tvmc_estimate", "tvmc_sr_solve", "tvmc_sde_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (tvmc_\w+)", out))
    assert set(_declared()) <= exported


def test_binding_names_match_the_header():
    from paper_2506_23928_amd import tvmc
    assert sorted(tvmc.EXPORTED) == _declared()


def test_struct_layouts_match_the_header(tmp_path):
    from paper_2506_23928_amd import tvmc
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "tvmc.h"\nint main(){'
                    'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(tvmc_problem), offsetof(tvmc_problem, jump_rate),'
                    'sizeof(tvmc_config), offsetof(tvmc_config, dt), offsetof(tvmc_config, precision),'
                    'offsetof(tvmc_config, seed), offsetof(tvmc_config, unravelling), offsetof(tvmc_config, use_graph),'
                    'offsetof(tvmc_config, sampler_chains),'
                    'sizeof(tvmc_ansatz));'
                    ' return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(prog)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    P, C, A = tvmc.tvmc_problem, tvmc.tvmc_config, tvmc.tvmc_ansatz
    want = [ctypes.sizeof(P), P.jump_rate.offset, ctypes.sizeof(C), C.dt.offset, C.precision.offset, C.seed.offset,
            C.unravelling.offset, C.use_graph.offset, C.sampler_chains.offset, ctypes.sizeof(A)]
    assert got == want


def test_configuration_checks_run_on_the_host():
    # tvmc_workspace_size validates the configuration without touching a device
    import numpy as np
    import pytest
    from paper_2506_23928_amd import tvmc
    pb = tvmc.Problem(np.zeros((4, 4)), 0.1, [(0, 0, 0.1)])
    an = tvmc.make_ansatz(tvmc.JASTROW, 0)
    lin = tvmc.make_config(2, 64, 8, 0.01, unravelling=tvmc.SSE_LINEAR)
    assert tvmc.tvmc_workspace_size(pb, an, lin) == tvmc.tvmc_workspace_size(pb, an, tvmc.make_config(2, 64, 8, 0.01))
    with pytest.raises(tvmc.TvmcError):
        tvmc.tvmc_workspace_size(pb, an, tvmc.make_config(2, 64, 8, 0.01, unravelling=2))
    # LJPHd: d in [0, N-1], parameter-space solve, exact int8 sums; the workspace grows with M
    lj = tvmc.make_ansatz(tvmc.LJPH, 1)
    assert tvmc.tvmc_workspace_size(pb, lj, tvmc.make_config(2, 64, 8, 0.01)) > 0
    for bad_an, bad_cfg in [(tvmc.make_ansatz(tvmc.LJPH, 4), tvmc.make_config(2, 64, 8, 0.01)),
                            (tvmc.make_ansatz(tvmc.LJPH, -1), tvmc.make_config(2, 64, 8, 0.01)),
                            (lj, tvmc.make_config(2, 64, 8, 0.01, solver=tvmc.SOLVER_SAMPLE_SPACE))]:
        with pytest.raises(tvmc.TvmcError):
            tvmc.tvmc_workspace_size(pb, bad_an, bad_cfg)
    # the int8 S-build sums n_samples products of magnitude up to (N - d - 1)^2 = 62^2 at N = 64,
    # d = 1, in int32: 2^19 * 3844 < 2^31 <= 2^20 * 3844
    pb64 = tvmc.Problem(np.zeros((64, 64)), 0.1, [(0, 0, 0.1)])
    ok = tvmc.make_config(1, 1 << 19, 64, 0.01, precision=tvmc.PREC_MFMA)
    assert tvmc.tvmc_workspace_size(pb64, lj, ok) > 0
    with pytest.raises(tvmc.TvmcError):
        tvmc.tvmc_workspace_size(pb64, lj, tvmc.make_config(1, 1 << 20, 64, 0.01, precision=tvmc.PREC_MFMA))
    # beyond N = 128 the distance sums enter as halves: at N = 192, d = 0 (LJH) up to 96^2 per
    # product, 232960 * 9216 < 2^31 <= 233024 * 9216 (n_samples a multiple of 64)
    pb192 = tvmc.Problem(np.zeros((192, 192)), 0.1, [(0, 0, 0.1)])
    ljh = tvmc.make_ansatz(tvmc.LJPH, 0)
    assert tvmc.tvmc_workspace_size(pb192, ljh, tvmc.make_config(1, 232960, 8, 0.01, precision=tvmc.PREC_MFMA)) > 0
    with pytest.raises(tvmc.TvmcError):
        tvmc.tvmc_workspace_size(pb192, ljh, tvmc.make_config(1, 233024, 8, 0.01, precision=tvmc.PREC_MFMA))
    # SNR solve: parameter space, M <= 2176, tau >= 0; it adds workspace (complex for the RBM)
    snr = tvmc.make_config(2, 64, 8, 0.01, regulariser=tvmc.REG_SNR)
    plain = tvmc.make_config(2, 64, 8, 0.01)
    assert tvmc.tvmc_workspace_size(pb, an, snr) > tvmc.tvmc_workspace_size(pb, an, plain)
    rbm = tvmc.make_ansatz(tvmc.RBM, 2)
    assert tvmc.tvmc_workspace_size(pb, rbm, snr) > tvmc.tvmc_workspace_size(pb, rbm, plain)
    assert tvmc.tvmc_workspace_size(pb64, an, snr) > 0          # M = 2080
    with pytest.raises(tvmc.TvmcError):
        tvmc.tvmc_workspace_size(pb64, tvmc.make_ansatz(tvmc.RBM, 40), snr)   # M = 64 + 40 + 2560 > 2176
    for bad_an, bad_cfg in [(an, tvmc.make_config(2, 64, 8, 0.01, regulariser=tvmc.REG_SNR, snr_tau=-1.0)),
                            (an, tvmc.make_config(2, 64, 8, 0.01, regulariser=tvmc.REG_SNR,
                                                  solver=tvmc.SOLVER_SAMPLE_SPACE)),
                            (an, tvmc.make_config(2, 64, 8, 0.01, regulariser=2))]:
        with pytest.raises(tvmc.TvmcError):
            tvmc.tvmc_workspace_size(pb, bad_an, bad_cfg)


def test_product_couplings_match_the_definition():
    # the library's host-side problem builder against brute-force sums (Eq. 10, Kac factor)
    import numpy as np
    from paper_2506_23928_amd.problem import kac_couplings
    n, alpha = 9, 1.5
    J = kac_couplings("obc", n, alpha)
    kac = sum(abs(i - j) ** -alpha for i in range(n) for j in range(i + 1, n)) / (n - 1)
    assert abs(J[0, 3] - 3 ** -alpha / kac) < 1e-14 and J[4, 4] == 0.0
    Jp = kac_couplings("pbc", 10, 1.0)
    assert abs(Jp[0, 9] - Jp[0, 1]) < 1e-15 and abs(Jp[0, 5] / Jp[0, 1] - 0.2) < 1e-14

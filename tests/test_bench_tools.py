"""CPU checks of the benchmark's host-side tooling: launch-class names of kernels, the rocprofv3 counter
summary (reference-copy scaling, set-up dispatches dropped) and the source-keyed traffic record."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("name,cls", [
    ("void cola::k_contract<cola::PolF32, 1, 4, false>(cola::PassArgs)", "contract_cols_f32"),
    ("void cola::k_contract<cola::PolBF16, 2, 2, true>(cola::PassArgs)", "contract_rows_bf16"),
    ("void cola::k_slab23<cola::SlabF64, true, false>(cola::SlabArgs)", "slab23_f64"),
    ("void cola::k_cg_update<float>(float*, float*, float const*, float const*, long)", "update_float"),
    ("cola::(anonymous namespace)::k_gemm2_t(cola::Gemm2Args)", "k_gemm2_t"),
    ("__amd_rocclr_copyBuffer", "other"),
])
def test_kernel_class(name, cls):
    assert bench.kernel_class(name) == cls


def _write_csv(path, rows):
    keys = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value", "Start_Timestamp",
            "End_Timestamp"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=keys)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(keys, r)))


def test_pmc_summary_scales_by_reference_copy(tmp_path, capsys):
    mul = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, " \
          "at::native::binary_internal::MulFunctor<float> > >"
    upd = "void cola::k_cg_update<float>(float*)"
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # set-up dispatch (dropped), elementwise reference, runtime copy (marker), two solver dispatches
    _write_csv(fetch, [(1, upd, 64, "FETCH_SIZE", 999.0, 0, 1000), (2, mul, 64, "FETCH_SIZE", 131072.0, 0, 1000),
                       (3, "__amd_rocclr_copyBuffer", 64, "FETCH_SIZE", 131072.0, 0, 1000),
                       (4, upd, 64, "FETCH_SIZE", 100.0, 0, 2000), (5, upd, 64, "FETCH_SIZE", 300.0, 0, 4000)])
    _write_csv(write, [(1, upd, 64, "WRITE_SIZE", 999.0, 0, 1000), (2, mul, 64, "WRITE_SIZE", 262144.0, 0, 1000),
                       (3, "__amd_rocclr_copyBuffer", 64, "WRITE_SIZE", 262144.0, 0, 1000),
                       (4, upd, 64, "WRITE_SIZE", 50.0, 0, 2000), (5, upd, 64, "WRITE_SIZE", 150.0, 0, 4000)])
    out = tmp_path / "traffic.json"
    bench.pmc_summary([str(fetch), str(write)], "c2", str(out))
    rec = json.load(open(out))["c2"]
    assert rec["scale"]["FETCH_SIZE"] == pytest.approx(2.0)
    assert rec["scale"]["WRITE_SIZE"] == pytest.approx(1.0)
    upd_rec = rec["kernels"]["update"]
    # averages over the two solver dispatches only: fetch 200 KiB x 2, write 100 KiB x 1
    assert upd_rec["bytes_per_launch_all_rhs_active"] == 1024 * (200 * 2 + 100)
    assert upd_rec["sources_sha1"] == bench.sources_digest("update")
    assert "update_float | 2 |" in capsys.readouterr().out


def test_measured_traffic_follows_active_rhs_and_sources(tmp_path, monkeypatch):
    rec = {"c2": {"scale": {}, "kernels": {"update": {"bytes_per_launch_all_rhs_active": 3200,
                                                      "sources_sha1": bench.sources_digest("update")}}}}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PMC_FILE", str(path))
    # 10 launches carrying 160 RHS*iterations of 32 RHS: half active on average
    assert bench.measured_traffic("c2", "update", 32, 160, 10) == 1600
    rec["c2"]["kernels"]["update"]["sources_sha1"] = "stale"
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("c2", "update", 32, 160, 10) is None


def test_measured_traffic_of_multi_iteration_launches(tmp_path, monkeypatch):
    """A fused launch record covers rhs_iters_per_dispatch RHS*iterations; traffic per launch follows the
    RHS*iterations the timed launches actually carried."""
    rec = {"c2": {"scale": {}, "kernels": {"cg_fused": {"bytes_per_launch_all_rhs_active": 1024 * 400,
                                                        "rhs_iters_per_dispatch": 1024,
                                                        "sources_sha1": bench.sources_digest("cg_fused")}}}}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PMC_FILE", str(path))
    # 4 launches carrying 2048 RHS*iterations: 512 each at 400 bytes
    assert bench.measured_traffic("c2", "cg_fused", 32, 2048, 4) == 512 * 400
    assert bench.source_kind("k_fused_cg") == "cg_fused" and bench.source_kind("contract_cols_f32") == "contract"
    assert bench.kernel_class("cola::(anonymous namespace)::k_fused_cg<2>(cola::FusedCgArgs)") == "k_fused_cg"


def test_unrolled_baselines_match_oracle_on_cpu():
    """The comparison baseline of the backward-memory experiment (plain-torch CG recorded by autograd) is
    itself checked against the oracle on the CPU: its Kronecker MVM entry by entry, its converged solve,
    its SLQ estimate with the same probes and steps, and its gradients on a well-conditioned operator
    (where reverse mode through CG is stable) against the closed forms."""
    import numpy as np
    import torch
    import workloads as wl
    from oracle import direct, grad, kron, slq
    pts = wl.config2(m=6, nrhs=1).systems[0].points
    facs = [wl.rbf_kernel(p, 0.3) for p in pts]
    s2 = 1.0
    rng = np.random.default_rng(5)
    V = rng.standard_normal((2, 216))
    K = [torch.tensor(f) for f in facs]
    got = bench.torch_kron3_mvm(K, s2, torch.tensor(V).reshape(2, 6, 6, 6)).reshape(2, -1).numpy()
    np.testing.assert_allclose(got, kron.mvm([facs], V, s2), rtol=1e-13, atol=1e-13)
    ell = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(s2, dtype=torch.float64, requires_grad=True)
    B = rng.standard_normal((2, 216))
    W = rng.standard_normal((2, 216))
    x, _, _ = bench.unrolled_cg(bench._rbf_factors([torch.tensor(p) for p in pts], ell), sig,
                                torch.tensor(B).reshape(2, 6, 6, 6), 60)
    (torch.tensor(W).reshape(2, 6, 6, 6) * x).sum().backward()
    X = direct.kron_eig_solve(facs, B, s2)
    L = direct.kron_eig_solve(facs, W, s2)
    np.testing.assert_allclose(x.detach().reshape(2, -1).numpy(), X, rtol=0, atol=1e-10 * np.abs(X).max())
    dfac, _, ds2 = grad.grad_kron([facs], X, L)
    dell = sum(grad.rbf_lengthscale_grad(dfac[0][k], facs[k], pts[k], 0.3) for k in range(3))
    assert abs(float(ell.grad) - dell) <= 1e-8 * abs(dell)
    assert abs(float(sig.grad) - ds2) <= 1e-8 * abs(ds2)
    Z = wl.rademacher_probes(rng, 3, 216)
    ld = bench.unrolled_slq_logdet(K, s2, torch.tensor(Z).reshape(3, 6, 6, 6), 7)
    ref = slq.slq_logdet(lambda M: kron.mvm([facs], M, s2), Z, 7)
    assert abs(float(ld) - ref) <= 1e-10 * abs(ref)


def test_class_model_bytes_per_engine_layout():
    """Algorithmic bytes per element of the three-GEMM launch classes (one term, three 256-wide
    modes), each following its reads and writes: 60 B per element and iteration with x in the
    update or split over the middle and last passes, 56 B with x in the direction pass (which
    holds p_old already, so the update no longer reads p)."""
    n, dims = 256 ** 3, [256, 256, 256]
    by = {}
    for deferral in (None, "first", "split"):
        by[deferral] = {c: bench.class_model(c, "bf16x3", n, dims, 1, False, deferral)[1] / n
                        for c in ("gemm_mode3", "gemm_mode2", "gemm_mode1", "update")}
    assert by[None] == {"gemm_mode3": 16, "gemm_mode2": 8, "gemm_mode1": 12, "update": 24}
    assert by["first"] == {"gemm_mode3": 24, "gemm_mode2": 8, "gemm_mode1": 12, "update": 12}
    assert by["split"] == {"gemm_mode3": 16, "gemm_mode2": 14, "gemm_mode1": 18, "update": 12}
    assert sum(by[None].values()) == 60 and sum(by["split"].values()) == 60
    assert sum(by["first"].values()) == 56
    # the diagonal adds its read to the last pass; FLOPs count the six BF16x3 products per useful one
    fl, b = bench.class_model("gemm_mode1", "bf16x3", n, dims, 1, True, "split")
    assert b / n == 22 and fl == 2.0 * n * 256 * 6

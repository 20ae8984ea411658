"""The build entry point that allocates nothing (hfx_build_2e_noalloc_dev,
per-build scratch in the library's fixed device array) against the
existing hfx_build_2e_dev on the same inputs, through the C ABI."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _pair(ctx, D, cj, ck, s, torch):
    dD = torch.tensor(D, device="cuda")
    ref, out = torch.empty_like(dD), torch.full_like(dD, np.nan)
    st_ref = ctx.build_2e_dev(dD.data_ptr(), cj, ck, ref.data_ptr(), s, stats=True)
    st_out = ctx.build_2e_noalloc_dev(dD.data_ptr(), cj, ck, out.data_ptr(), s, stats=True)
    torch.cuda.synchronize()
    return ref, out, st_ref, st_out


def test_noalloc_equals_build_2e_dev_two_calls_in_a_row():
    """Two calls in a row on one GPU, the second with a smaller molecule (so
    the fixed array still holds the first call's larger accumulator): both
    equal hfx_build_2e_dev's result; persistent and per-wave launch forms
    (queue counters in the array), FP64 and mixed precision."""
    import torch
    from paper_1708_00033_amd import hfx
    s = torch.cuda.current_stream().cuda_stream
    cases = [(W.water_cluster(16, 77), 5, hfx.HFX_PREC_FP64, (8192, 1, 1, -1), 2.0, 1.0),
             (W.water_cluster(4, 41), 6, hfx.HFX_PREC_FP64, (2048, 1, 2, -1), 1.0, 0.0),
             (W.water_cluster(16, 78), 7, hfx.HFX_PREC_MIXED, (32768, 0, 0, -1), 2.0, 1.0),
             (W.dimer_config(), 8, hfx.HFX_PREC_MIXED, (256, 0, 0, 1), 0.0, -1.0)]
    for mol, seed, prec, tune, cj, ck in cases:
        ctx = hfx.Context(precision=prec).load(mol)
        ctx.set_class_tuning(-1, *tune)
        D = W.random_orthonormal_density(mol.nbf, mol.nocc, seed)
        ref, out, st_ref, st_out = _pair(ctx, D, cj, ck, s, torch)
        assert torch.isfinite(out).all()
        assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item(), (mol.name, prec)
        assert (st_out.quartets_fp64, st_out.quartets_fp32) == (st_ref.quartets_fp64, st_ref.quartets_fp32)


def test_noalloc_batch_and_size_limit():
    """A batch (ragged accumulator in the array) equals the eager build; a
    system beyond the array's size is refused before anything is launched."""
    import torch
    from paper_1708_00033_amd import hfx
    s = torch.cuda.current_stream().cuda_stream
    mols = [W.water_cluster(3, 91), W.water_cluster(1, 92), W.water_cluster(5, 93)]
    ctx = hfx.Context().load_batch(mols)
    nbf, nocc, off, tot = ctx.layout
    D = np.concatenate([W.random_orthonormal_density(int(n), int(o), 10 + i).ravel()
                        for i, (n, o) in enumerate(zip(nbf, nocc))])
    ref, out, _, _ = _pair(ctx, D, 2.0, 1.0, s, torch)
    assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item()
    big = hfx.Context().load(W.water_cluster(80, 3))   # 1520 basis functions: 37 MB of scratch
    dD = torch.zeros((big.nbf, big.nbf), dtype=torch.float64, device="cuda")
    dG = torch.full_like(dD, 7.0)
    with pytest.raises(hfx.HfxError) as e:
        big.build_2e_noalloc_dev(dD.data_ptr(), 2.0, 1.0, dG.data_ptr(), s)
    assert e.value.status == hfx.HFX_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert (dG == 7.0).all()

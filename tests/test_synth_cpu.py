"""The seeded input generators (no method arithmetic): the fill routines that
write a workload straight into a tensor must give the host generator's
stored values bit for bit (run here with CPU tensors; the device runs the same
elementwise FP64 operations)."""
import numpy as np
import torch

import synth


def test_bump_fill_matches_host_generator():
    w = synth.bump_field(5, m=700, n=300)
    for dtype, chunk in ((torch.float64, 128), (torch.float32, 97)):
        out = torch.empty((700, 300), dtype=dtype)
        synth.bump_fill(5, out, rows_per_chunk=chunk)
        want = synth.quantize(w.X, "f64" if dtype == torch.float64 else "f32")[0]
        assert np.array_equal(out.numpy(), want), dtype
    out = torch.empty((700, 300), dtype=torch.bfloat16)
    synth.bump_fill(5, out, rows_per_chunk=256)
    bits = out.view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(bits, synth.quantize(w.X, "bf16")[0])


def test_parametric_fill_matches_host_rows():
    pf = synth.parametric_field(0, grid=40, n=64)
    out = torch.empty((pf.m, pf.n), dtype=torch.float32)
    pf.fill_device(out, rows_per_chunk=400)
    assert np.array_equal(out.numpy(), synth.quantize(pf.full(), "f32")[0])

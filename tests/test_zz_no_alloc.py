"""The renderer forward that allocates nothing (gsim_raster_forward_noalloc: scratch in
the library's static device array) against the renderer forward with its own workspace
(gsim_raster_forward), through the C-ABI: bitwise equal images on two calls in a row,
the second with a smaller mesh and image (the static scratch keeps the first call's
contents), in FP32 and FP64; sizes beyond the array are refused before any launch; a
triangle with an index out of range covers nothing."""
import numpy as np
import pytest

from paper_2104_02646_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _view(n, H, Wd):
    b = W.cloth(31, n=n, size=1.0, height=1.0)
    eye, target, up = np.array([0.5, 2.2, 2.6]), np.array([0.5, 1.0, 0.5]), np.array([0.0, 1.0, 0.0])
    fwd = (target - eye) / np.linalg.norm(target - eye)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    Rm = np.stack([right, down, fwd])
    K = np.array([[1.1 * Wd, 0, Wd / 2], [0, 1.1 * Wd, H / 2], [0, 0, 1.0]])
    return b, K @ np.concatenate([Rm, (-Rm @ eye)[:, None]], 1)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_forward_equals_workspace_forward(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_02646_amd import gsim
    gsim.load()
    rng = np.random.default_rng(8)
    # first a mesh of 1682 triangles (more than one 512-triangle chunk) at 96x104, then a
    # smaller one at 40x48: the second call runs over what the first left in the scratch
    for n, H, Wd in ((30, 96, 104), (8, 40, 48)):
        b, P = _view(n, H, Wd)
        x = gsim.soa(b.X + rng.normal(0, 0.01, b.X.shape), dtype=dtype)
        ref = gsim.Renderer(b.tris, b.np, H, Wd, dtype).forward(x, P, 1.5)
        tris = torch.as_tensor(np.ascontiguousarray(b.tris, np.int32), device="cuda")
        out = torch.full((H, Wd), float("nan"), dtype=dtype, device="cuda")
        gsim.raster_forward_noalloc(tris, b.np, H, Wd, x, P, 1.5, out)
        torch.cuda.synchronize()
        print("%s %d triangles at %dx%d: coverage %.3f, max |diff| %.1e" % (
            dtype, len(b.tris), H, Wd, float(ref.mean()), float((out - ref).abs().max())))
        assert float(ref.mean()) > 0.01
        assert torch.equal(out, ref)


def test_noalloc_limits_and_bad_indices():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_02646_amd import gsim
    gsim.load()
    b, P = _view(8, 40, 48)
    x = gsim.soa(b.X)
    out = torch.zeros(40, 48, device="cuda")
    tris = torch.as_tensor(np.ascontiguousarray(b.tris, np.int32), device="cuda")
    # an image whose transmittance alone exceeds the scratch: refused, nothing launched
    big = torch.zeros(4096, 4096, device="cuda")
    with pytest.raises(gsim.GsimError) as e:
        gsim.raster_forward_noalloc(tris, b.np, 4096, 4096, x, P, 1.5, big)
    assert e.value.code == gsim.GSIM_E_WORKSPACE
    with pytest.raises(ValueError):  # an output smaller than the image: refused by the binding
        gsim.raster_forward_noalloc(tris, b.np, 4096, 4096, x, P, 1.5, out)
    # the last triangle with a corner index just past the vertices (it stays inside the
    # scratch even if it were read): the image equals the mesh without that triangle
    bad = b.tris.copy()
    bad[-1, 2] = b.np
    gsim.raster_forward_noalloc(torch.as_tensor(bad, device="cuda"), b.np, 40, 48, x, P, 1.5, out)
    ref = gsim.Renderer(b.tris[:-1], b.np, 40, 48).forward(x, P, 1.5)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)

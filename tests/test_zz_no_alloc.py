"""The no-allocation entry point (she_debug_normals_noalloc) against the
allocating one (she_debug_normals), through the C ABI: two calls in a row,
the second with fewer numbers, each bit for bit equal to the allocating
call's numbers; a count above the fixed staging array is refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def she():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_12157_amd import she as mod
    mod.load()
    return mod


def test_noalloc_normals_equal_the_allocating_entry_point(she):
    calls = [(7, 3, 0, 123456, 1001, she.NOALLOC_MAX_NORMALS, she.F32),   # fills the whole array
             (9, 1, 1, 2 ** 33 + 5, 77, 1000, she.F64),                   # then a smaller call
             (0, 0, 0, 0, 0, 5, she.F32)]
    for seed, real, tag, step, face0, count, prec in calls:
        got = she.debug_normals_noalloc(seed, real, tag, step, face0, count, prec)
        want = she.debug_normals(seed, real, tag, step, face0, count, prec)
        assert got.shape == (count,)
        np.testing.assert_array_equal(got, want)
        assert np.all(np.isfinite(got)) and np.std(got) > 0.5
    with pytest.raises(she.SheError) as e:
        she.debug_normals_noalloc(0, 0, 0, 0, 0, she.NOALLOC_MAX_NORMALS + 1, she.F32)
    assert e.value.status == she.EINVAL
    assert she.debug_normals_noalloc(0, 0, 0, 0, 0, 0, she.F32).shape == (0,)

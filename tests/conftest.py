import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


# ---- GPU fixtures ----------------------------------------------------------------------

def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="session")
def gpu_ctx():
    _need_gpu()
    import torch
    from paper_2010_08735_amd import bh
    torch.cuda.init()
    ctx = bh.bh_create(0, 0)
    yield ctx
    torch.cuda.synchronize()
    bh.bh_destroy(ctx)


@pytest.fixture(scope="session")
def gpu_tables(gpu_ctx):
    from paper_2010_08735_amd import bh
    t = bh.bh_precompute_tables(gpu_ctx, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
    return t


@pytest.fixture(scope="session")
def orc_tables(orc):
    return orc.Tables(512, 64, 32)


@pytest.fixture(scope="session")
def orc_ctable(orc):
    """The oracle's colour-shift table at the library's node counts (FP64)."""
    return orc.cshift_table(*orc.CSHIFT_DIMS)


@pytest.fixture(scope="session")
def small_scene(gpu_ctx, orc):
    """20 000 seeded stars in a 6 x 256^2 FP16 map (GPU) and the oracle's map."""
    from paper_2010_08735_amd import bh, scenes
    field = scenes.star_field(20000, 0)
    n0 = 256
    h = gpu_star_map(gpu_ctx, field, n0, bh.BH_TEXEL_FP16)
    return field, n0, h, orc.cubemap(field, n0)


@pytest.fixture(scope="session")
def big_field_scene(gpu_ctx, orc):
    """One million seeded stars in a 6 x 2048^2 FP16 map (GPU) and the oracle's map."""
    from paper_2010_08735_amd import bh, scenes
    field = scenes.star_field(1_000_000, 1)
    n0 = 2048
    h = gpu_star_map(gpu_ctx, field, n0, bh.BH_TEXEL_FP16)
    return field, n0, h, orc.cubemap(field, n0)


def gpu_star_map(ctx, field, n0, fmt=0):
    import torch
    from paper_2010_08735_amd import bh
    d = torch.from_numpy(field.dirs).cuda()
    i = torch.from_numpy(field.intensity).cuda()
    t = torch.from_numpy(field.temperature).cuda()
    h = bh.bh_build_stars(ctx, d.data_ptr(), i.data_ptr(), t.data_ptr(), len(field), n0, fmt,
                          bh.current_stream())
    torch.cuda.synchronize()
    return h

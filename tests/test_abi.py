"""The C ABI library on the host: it loads, exports every function the header
declares, validates parameters before touching the GPU, and seeds particles
bit-identically to the shared input generator."""
import ctypes

import numpy as np
import pytest

import lbm_inputs
from paper_2308_16597_amd import lbm


def test_every_declared_function_is_exported():
    names = lbm.declared_functions()
    assert len(names) >= 17
    so = ctypes.CDLL(lbm.LIB_PATH)
    for n in names:
        assert hasattr(so, n), n


def test_abi_version_and_defaults():
    assert lbm.lbm_abi_version() == 4
    p = lbm.lbm_params_default()
    assert (p.abi_version, p.nx, p.ny, p.periodic_x, p.periodic_y, p.storage) == (4, 64, 64, 1, 0, 0)
    assert p.streaming == lbm.STREAMING["two_sets"]
    assert (p.rho0, p.a_T, p.rep_eps, p.rep_range, p.repulsion) == (1.0, -2.0, 1e-3, 3.0, 1)
    assert tuple(p.side_T) == (0.0, 0.0)


def test_params_struct_matches_the_header_layout():
    # the offsets of the fields added last, as the C compiler lays them out
    assert lbm.LbmParams.side_T.offset == 232 and lbm.LbmParams.streaming.offset == 248
    assert ctypes.sizeof(lbm.LbmParams) == 256


@pytest.mark.parametrize("bad", [dict(nx=4), dict(ny=70000), dict(periodic_x=2), dict(storage=9),
                                 dict(nu=0.0), dict(alpha=-1.0), dict(s_q=2.5), dict(a_T=-5.0),
                                 dict(max_particles=-1),
                                 dict(max_particles=10, max_diameter=2.0),
                                 dict(max_particles=10, max_diameter=12.0, periodic_y=1),
                                 dict(nx=16, max_particles=10, max_diameter=14.0),
                                 dict(gravity=float("inf")), dict(abi_version=7),
                                 dict(abi_version=3), dict(periodic_x=0, side_T=(float("nan"), 0.0)),
                                 dict(streaming=2)])
def test_invalid_parameters_rejected_on_the_host(bad):
    p = lbm.lbm_params_default(**bad)
    assert lbm.lbm_bytes_required(p) == 0
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p)
    assert e.value.rc == lbm.LBM_EINVAL
    assert lbm.lbm_last_error()


def test_in_place_streaming_halves_the_population_memory():
    kw = dict(nx=4000, ny=4000, max_particles=4800, max_diameter=20.0)
    two = lbm.lbm_bytes_required(lbm.lbm_params_default(**kw))
    one = lbm.lbm_bytes_required(lbm.lbm_params_default(streaming="in_place", **kw))
    pops = 14 * 4000 * 4096 * 8
    assert two - one > 0.85 * pops and one < 0.6 * two


def test_bytes_required_grows_with_the_lattice_and_storage():
    small = lbm.lbm_bytes_required(lbm.lbm_params_default(nx=256, ny=256))
    big = lbm.lbm_bytes_required(lbm.lbm_params_default(nx=512, ny=256))
    half = lbm.lbm_bytes_required(lbm.lbm_params_default(nx=512, ny=256, storage="shift_bf16"))
    assert 0 < small < big and half < big
    # 4000^2 in FP64 with 4800 particles: two time levels of 14 arrays dominate
    p = lbm.lbm_params_default(nx=4000, ny=4000, max_particles=4800, max_diameter=20.0)
    assert 2 * 14 * 4000 * 4000 * 8 < lbm.lbm_bytes_required(p) < 4.2e9


@pytest.mark.parametrize("nx,ny,n,d,gap,seed", [(256, 256, 20, 12.0, 1.0, 1),
                                                (4000, 4000, 4800, 20.0, 1.0, 2),
                                                (300, 200, 120, 9.0, 2.0, 77)])
def test_rsa_seed_is_bit_identical_to_the_input_generator(nx, ny, n, d, gap, seed):
    a = lbm.lbm_rsa_seed(nx, ny, n, d, gap, seed)
    b = lbm_inputs.rsa_particles(nx, ny, n, d, gap, seed)
    np.testing.assert_array_equal(a, b)


def test_rsa_seed_reports_infeasible_packing():
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_rsa_seed(32, 32, 40, 10.0, 1.0, 1)
    assert e.value.rc == lbm.LBM_ESEED


def test_step_many_rejects_empty_run_lists_on_the_host():
    f = lbm._lib.lbm_step_many
    assert f(None, 0, None, None) == lbm.LBM_EINVAL
    hs = (ctypes.c_void_p * 2)(None, None)
    ns = np.zeros(2, dtype=np.int32)
    assert f(ctypes.cast(hs, ctypes.c_void_p), 2, ns.ctypes.data, None) == lbm.LBM_EINVAL
    assert "null handle" in lbm.lbm_last_error(None)


def links_wave_lds(nwin):
    """LDS of one particle of the link collection: the owner-map window and
    the 12 N - 12 slots as 4-byte words (rounded to 8 bytes), then the
    compacted list of 8-byte links."""
    slots = 12 * nwin - 12
    return ((nwin * nwin + slots) * 4 + 7) // 8 * 8 + slots * 8


@pytest.mark.parametrize("d,n", [(10.0, 64000), (20.0, 4800), (40.0, 4800), (46.0, 2000), (60.0, 5000),
                                 (80.0, 1500), (96.0, 1100), (96.0, 500), (30.0, 10)])
def test_link_collection_lds_stays_within_64_kib(d, n):
    """The collection's dynamic LDS per block is bounded for every diameter
    the parameters accept: four particles' windows share a block only while
    they fit in 64 KiB, else each particle takes a block of its own."""
    p = lbm.lbm_params_default(nx=4096, ny=4096, max_particles=n, max_diameter=d)
    got = lbm.lbm_collect_lds_bytes(p)
    nwin = int(d) + 4
    one = links_wave_lds(nwin)
    assert got in (one, 4 * one)
    assert got <= 65536
    # the shared block is kept whenever it fits
    if nwin < 32 and 4 * one <= 65536:
        assert got == 4 * one


def test_collect_lds_of_invalid_or_particle_free_parameters_is_zero():
    assert lbm.lbm_collect_lds_bytes(lbm.lbm_params_default(nx=4)) == 0
    assert lbm.lbm_collect_lds_bytes(lbm.lbm_params_default()) == 0


def test_budget_admission():
    p = lbm.lbm_params_default(nx=512, ny=256, max_particles=40, max_diameter=12.0)
    need = lbm.lbm_bytes_required(p)
    assert need > 0
    assert lbm.lbm_check_budget(p, need) == lbm.LBM_OK
    assert lbm.lbm_check_budget(p, need - 1) == lbm.LBM_EBUDGET
    assert "budget" in lbm.lbm_last_error()
    assert lbm.lbm_check_budget(lbm.lbm_params_default(nx=4), 1 << 40) == lbm.LBM_EINVAL


def test_arena_smaller_than_the_run_is_a_budget_error():
    # rejected on the host, before any device call: the size is checked first
    p = lbm.lbm_params_default(nx=64, ny=64)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create_in_arena(p, 1 << 20, lbm.lbm_bytes_required(p) - 256)
    assert e.value.rc == lbm.LBM_EBUDGET


def test_create_without_a_gpu_is_a_device_error():
    """With no GPU the library fails loudly at creation: a device error that
    names the allocation, and no handle (there is no CPU path)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    p = lbm.lbm_params_default(nx=64, ny=64)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p)
    assert e.value.rc == lbm.LBM_EDEVICE
    assert "hipMalloc" in str(e.value) and "hipMalloc" in lbm.lbm_last_error()

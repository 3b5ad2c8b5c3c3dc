"""Host logic of the profile summaries: kernel names as the library's profiler uses them,
and HBM bytes per launch scaled by a plain copy of known size (synthetic counter files)."""
import csv
import json

import pytest

from paper_2009_06725_amd.rocprof_summary import short_name, traffic


@pytest.mark.parametrize("demangled,name", [
    ("void scvs::(anonymous namespace)::k_vstep<3, float>(scvs::MeshArgs, ...)", "k_vstep32"),
    ("void scvs::(anonymous namespace)::k_vstep<3, double>(scvs::MeshArgs, ...)", "k_vstep"),
    ("void scvs::(anonymous namespace)::k_full<3, 0, false, float, true, HIP_vector_type<double, 2u> >(...)",
     "k_full_apply32"),
    ("void scvs::(anonymous namespace)::k_full<3, 1, true, double, false, HIP_vector_type<double, 2u> >(...)",
     "k_full_resid"),
    ("void scvs::(anonymous namespace)::k_pstep<HIP_vector_type<double, 2u>, float>(...)", "k_pstep32"),
    ("void scvs::(anonymous namespace)::k_pstep<HIP_vector_type<float, 2u>, double>(...)", "k_pstep"),
    ("void scvs::(anonymous namespace)::k_pinit<HIP_vector_type<double, 2u>, float>(...)", "k_pinit32"),
    ("void scvs::(anonymous namespace)::k_lag_dots<HIP_vector_type<double, 2u> >(scvs::KArgs, int, int)",
     "k_lag_dots"),
    ("void scvs::(anonymous namespace)::k_dots<1>(...)", "k_dots1"),
    ("void scvs::(anonymous namespace)::k_mg_step_sell<float, 3, true, 0>(...)", "k_mgv_smooth0"),
    ("void scvs::(anonymous namespace)::k_mg_step_sell<float, 3, true, 1>(...)", "k_mgv_resid0"),
    ("void scvs::(anonymous namespace)::k_mg_step_sell<double, 1, false, 0>(...)", "k_mgp_smooth0"),
    ("void scvs::(anonymous namespace)::k_mg_step<float, 3, true, 0>(...)", "k_mgv_smooth"),
    ("void scvs::(anonymous namespace)::k_mg_step_sell4<3, true, 0>(...)", "k_mgv_smooth0"),
    ("void scvs::(anonymous namespace)::k_mg_step_sell2<1, false, 1>(...)", "k_mgp_resid0"),
    ("void scvs::(anonymous namespace)::k_mg_step_split<float, 1, false, 1>(...)", "k_mgp_resid"),
    ("void scvs::(anonymous namespace)::k_full_sell<3, HIP_vector_type<double, 2u> >(...)", "k_full_apply32"),
    ("void scvs::(anonymous namespace)::k_vinit_sell<3, HIP_vector_type<double, 2u> >(...)", "k_vinit32"),
    ("__amd_rocclr_copyBuffer", "__amd_rocclr_copyBuffer"),
])
def test_short_names(demangled, name):
    assert short_name(demangled) == name


def _write(dirpath, counter, rows):
    dirpath.mkdir(parents=True, exist_ok=True)
    with open(dirpath / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, v in rows:
            w.writerow({"Kernel_Name": k, "Grid_Size": 256, "Counter_Name": counter, "Counter_Value": v})


def test_sliced_kernel_on_a_coarse_level(tmp_path):
    """A sliced-row multigrid kernel's largest grid is level 0; smaller grids are coarse levels."""
    copy = "__amd_rocclr_copyBuffer"
    nbytes = 1 << 20
    _write(tmp_path / "cf", "FETCH_SIZE", [(copy, nbytes / 1024 / 2)])
    _write(tmp_path / "cw", "WRITE_SIZE", [(copy, nbytes / 1024)])
    k = "void scvs::(anonymous namespace)::k_mg_step_sell2<1, false, 0>(...)"
    for d, c in (("f", "FETCH_SIZE"), ("w", "WRITE_SIZE")):
        (tmp_path / d).mkdir()
        with open(tmp_path / d / "run_counter_collection.csv", "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
            w.writeheader()
            w.writerow({"Kernel_Name": k, "Grid_Size": 4096, "Counter_Name": c, "Counter_Value": 10.0})
            w.writerow({"Kernel_Name": k, "Grid_Size": 512, "Counter_Name": c, "Counter_Value": 1.0})
    r = traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"), nbytes,
                str(tmp_path / "t.json"))
    assert r["dispatches"] == {"k_mgp_smooth0": 1, "k_mgp_smooth": 1}
    assert r["bytes_per_launch"]["k_mgp_smooth0"] == pytest.approx((20.0 + 10.0) * 1024)


def test_traffic_scaling(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    nbytes = 1 << 20
    # the copy's counters read half of the bytes fetched and all of the bytes written (in KiB)
    _write(tmp_path / "cf", "FETCH_SIZE", [(copy, nbytes / 1024 / 2)] * 3)
    _write(tmp_path / "cw", "WRITE_SIZE", [(copy, nbytes / 1024)] * 3)
    k32 = "void scvs::(anonymous namespace)::k_vstep<3, float>(...)"
    # two dispatches of one kernel: fetch 100 and 300 KiB counted, write 50 KiB each
    _write(tmp_path / "f", "FETCH_SIZE", [(k32, 100.0), (k32, 300.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [(k32, 50.0), (k32, 50.0)])
    out = tmp_path / "t.json"
    r = traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"), nbytes,
                str(out))
    assert r["calibration"]["fetch_factor"] == pytest.approx(0.5)
    assert r["calibration"]["write_factor"] == pytest.approx(1.0)
    # mean fetch 200 KiB counted -> 400 KiB real; write 50 KiB
    assert r["bytes_per_launch"]["k_vstep32"] == pytest.approx((400.0 + 50.0) * 1024)
    assert r["dispatches"]["k_vstep32"] == 2
    assert json.load(open(out))["source_hash"] == r["source_hash"]

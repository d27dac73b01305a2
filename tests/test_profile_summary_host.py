"""Counter-summary helpers on the host: calibrated traffic from synthetic
rocprofv3 counter files, and its invalidation when the kernel sources change."""

import json
import os

from paper_2606_17212_amd import profile_summary as ps

K = "k_composite<8,16,16,0,false,256>"


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (name, v) in enumerate(rows):
            f.write(f'{i},"{name}",{counter},{v}\n')


def test_traffic_record_scales_by_the_copy_and_checks_sources(tmp_path):
    copy = 256 << 20
    kname = "void dgs::k_composite<8, 16, 16, 0, false, 256>(dgs::CompositeArgs)"
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>(int)"
    # the copy's FETCH reads half its bytes (factor 2), WRITE reads all of it (factor 1)
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(kname, 1000.0), (kname, 1200.0), (neg, copy / 2048), ("other", 7.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(kname, 500.0), (neg, copy / 2048), (neg, copy / 2048)])
    rec = ps.traffic_record(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), K, "wl", copy, "cmd")
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["fetch_bytes"] == 1100.0 * 1024 * 2 and rec["write_bytes"] == 500.0 * 1024
    root = tmp_path / "root"
    os.makedirs(root / "profiles")
    with open(ps.traffic_path(str(root), "wl"), "w") as f:
        json.dump(rec, f)
    assert ps.measured_traffic(K, "wl", str(root)) == round(rec["traffic_bytes"])
    assert ps.measured_traffic("k_composite<8,16,16,0,true,256>", "wl", str(root)) is None
    assert ps.measured_traffic("k_composite<8,16,16,0,false,128>", "wl", str(root)) is None
    assert ps.measured_traffic(K, "other_workload", str(root)) is None
    rec["sources_sha256"] = "0" * 64  # as if the kernel changed after the counters were taken
    with open(ps.traffic_path(str(root), "wl"), "w") as f:
        json.dump(rec, f)
    assert ps.measured_traffic(K, "wl", str(root)) is None

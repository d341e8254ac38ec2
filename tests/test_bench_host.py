"""Host-side arithmetic of the benchmark: the roofline's algorithmic byte
counts and the conversion of rocprofv3 byte counters into traffic files."""
import csv
import json

import numpy as np

import bench


class _Model:
    def __init__(self, n_tets, n_species, n_realizations):
        self.n_tets, self.n_species, self.n_realizations = n_tets, n_species, n_realizations


class _Sim:
    def __init__(self, counts):
        self.c = counts  # [Rz][S][T]

    def get_counts(self, species, realization=0):
        assert species is None
        return self.c[realization]


def test_scan_bytes_by_hand():
    # 2 species, 70 tets (Tp = 72, 18 groups, map row 18 -> 32 bytes), 2 realizations
    T, S = 70, 2
    c = np.zeros((2, S, T), np.int32)
    c[0, 0, 0] = 3      # group 0 (lane 0), species 0
    c[0, 1, 1] = 1      # group 0, species 1: tet 1 holds species 1 only
    c[0, 0, 69] = 2     # group 17 (lane 4), species 0
    c[1, 1, 17] = 5     # realization 1: group 4 (lane 1), species 1
    got = bench.scan_bytes([_Sim(c)], [_Model(T, S, 2)])
    map_bytes = 2 * (S * 32)   # read only: the map is not cleared
    vec = 4     # flagged four-tet vectors, per species: r0: s0 {0, 17}, s1 {0}; r1: s1 {4}
    tets = 4    # tets 0, 1, 69 and (r1) 17
    assert got == map_bytes + 32 * vec + (4 + 4 * S) * tets


def test_update_bytes():
    assert bench.update_bytes({"tets": 10, "additions": 7}, 3) == 10 * (4 + 12 + 64) + 9 * 7


def _csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, (name, v) in enumerate(rows, 1):
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def _pairs(scan, update, n):
    out = []
    for i in range(n):
        out += [("scan_kernel<3>(...)", scan(i)), ("update_kernel<false, 4>(...)", update(i))]
    return out


def test_write_traffic_scales_by_the_copy_kernel(tmp_path):
    # the copy kernel moves 1 GiB each way; its counters read half (fetch) and all (write) of it.
    # Earlier dispatches (tuning, replays) come first; the timing pass is the last 16 scan/update
    # pairs before the copies.
    gib_kib = (1 << 30) / 1024
    fetch = [("update_kernel<false, 4>(...)", 999.0)] * 3 + _pairs(lambda i: 999.0, lambda i: 999.0, 4)
    fetch += _pairs(lambda i: 100.0 + i, lambda i: 50.0, 16) + [("bandwidth_copy_kernel(...)", gib_kib / 2)] * 5
    write = [("update_kernel<false, 4>(...)", 999.0)] * 3 + _pairs(lambda i: 999.0, lambda i: 999.0, 4)
    write += _pairs(lambda i: 40.0, lambda i: 20.0 + i, 16) + [("bandwidth_copy_kernel(...)", gib_kib)] * 5
    _csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 16, ["cmd"], out_dir=str(tmp_path))
    scan = json.load(open(tmp_path / "scan_kernel_batched_traffic.json"))
    upd = json.load(open(tmp_path / "update_kernel_batched_traffic.json"))
    assert scan["scale"] == {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
    # the last 16 dispatches: fetch mean 107.5 KiB x 2, write 40 KiB x 1
    assert scan["fetch_bytes_per_launch"] == round(107.5 * 1024 * 2)
    assert scan["write_bytes_per_launch"] == 40 * 1024
    assert upd["fetch_bytes_per_launch"] == 50 * 1024 * 2
    assert upd["write_bytes_per_launch"] == round(27.5 * 1024)
    assert scan["kernel_sources"] == bench.kernel_source_hash() and scan["launches_averaged"] == 16
    assert not (tmp_path / "fused_kernel_batched_traffic.json").exists()


def test_write_traffic_refuses_a_run_without_the_timing_pass(tmp_path):
    # the last step dispatches before the copies are not scan/update pairs (e.g. a fused shape's
    # timing pass, whose kernel the counter run does not collect, after two-chain replays that end
    # on two updates): refused, no file written
    gib_kib = (1 << 30) / 1024
    rows = _pairs(lambda i: 100.0, lambda i: 50.0, 16) + [("update_kernel<false, 4>(...)", 50.0)]
    rows += [("bandwidth_copy_kernel(...)", gib_kib)] * 5
    _csv(tmp_path / "f.csv", "FETCH_SIZE", rows)
    _csv(tmp_path / "w.csv", "WRITE_SIZE", rows)
    import pytest

    with pytest.raises(SystemExit, match="scan/update pairs"):
        bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 16, ["cmd"], out_dir=str(tmp_path))
    assert not (tmp_path / "update_kernel_batched_traffic.json").exists()


def test_source_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    import os

    src = tmp_path / "paper_1512_03126_amd" / "csrc"
    src.mkdir(parents=True)
    for f, text in (("rdos_kernels.hip", "int a = 1; // x\n"), ("rdos_sampling.h", "/* y */ int b;"),
                    ("rdos_internal.h", "int c;")):
        (src / f).write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    (src / "rdos_kernels.hip").write_text("int   a = 1;   // another comment\n\n")
    assert bench.kernel_source_hash() == h0
    (src / "rdos_kernels.hip").write_text("int a = 2;\n")
    assert bench.kernel_source_hash() != h0
    assert os.path.exists(src / "rdos_internal.h")


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode != 0 and "one GPU" in r.stderr

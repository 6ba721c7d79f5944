"""The rocprofv3 summariser behind the roofline record: flop and byte
arithmetic on a small synthetic counter file."""

import csv
import json

import pytest

from paper_1909_01580_amd import counters

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


FLUX64 = "void hgks::k_flux_box<double, true, false>(double const*, ...)"
FLUX32 = "void hgks::k_flux_box<float, true, false>(float const*, ...)"


def test_flops_entry(tmp_path):
    rows = []
    for d in ("1", "2"):
        # counters split over two instances (summed), two dispatches (averaged)
        for name, v in (("SQ_WAVES", 50), ("SQ_INSTS_VALU", 1000), ("SQ_INSTS_VALU_FMA_F64", 300),
                        ("SQ_INSTS_VALU_MUL_F64", 100), ("SQ_INSTS_VALU_ADD_F64", 50),
                        ("SQ_INSTS_VALU_TRANS_F64", 5), ("GRBM_GUI_ACTIVE", 4000)):
            rows += [(d, FLUX64, name, v), (d, FLUX64, name, v)]
        rows.append((d, "void hgks::k_recon_box<double, false, true>(...)", "SQ_WAVES", 7))
    p = tmp_path / "pmc.csv"
    write_csv(p, rows)
    e = counters.flops_entry(str(p), "fp64")
    assert e["dispatches"] == 2
    assert e["waves_per_launch"] == 100
    assert e["valu_per_wave"] == 20
    # 64 lanes x (2 FMA + ADD + MUL + TRANS)
    assert e["flop_per_launch"] == 64 * (2 * 600 + 200 + 100 + 10)
    # 2000 VALU x 4 cycles over 1024 SIMDs x (8000 / 8) cycles
    assert e["issue_rate"] == pytest.approx(2000 * 4 / (1024 * 1000))


def test_traffic_uses_copy_calibration(tmp_path):
    mib = 64
    nb = mib << 20
    fetch = [("1", FLUX64, "FETCH_SIZE", 1000.0), ("2", FLUX32, "FETCH_SIZE", 500.0),
             # the copy reads half of what it fetches in this counter's units
             ("3", "__amd_rocclr_copyBuffer", "FETCH_SIZE", nb / 1024 / 2),
             ("4", "void at::native::elementwise_kernel<...>", "FETCH_SIZE", 3.0)]
    write = [("1", FLUX64, "WRITE_SIZE", 2000.0), ("2", FLUX32, "WRITE_SIZE", 1000.0),
             ("3", "__amd_rocclr_copyBuffer", "WRITE_SIZE", nb / 1024)]
    pf, pw = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(pf, fetch)
    write_csv(pw, write)
    out = tmp_path / "t.json"
    counters.main(["traffic", "--fetch", str(pf), "--write", str(pw), "--copy-mib", str(mib), "-o", str(out)])
    rec = json.loads(out.read_text())
    assert rec["fetch_factor"] == pytest.approx(2.0)
    assert rec["write_factor"] == pytest.approx(1.0)
    assert rec["fp64"]["bytes_per_launch"] == pytest.approx(1000 * 1024 * 2 + 2000 * 1024)
    assert rec["mixed"]["bytes_per_launch"] == pytest.approx(500 * 1024 * 2 + 1000 * 1024)
    assert rec["source_hash"] == counters.source_hash()


def test_pick_refuses_ambiguous(tmp_path):
    p = tmp_path / "x.csv"
    write_csv(p, [("1", FLUX64, "SQ_WAVES", 1), ("2", FLUX64.replace("true, false", "true, true"), "SQ_WAVES", 1)])
    with pytest.raises(SystemExit):
        counters.pick(counters.read_counters(str(p)), "k_flux_box", "<double")


def test_code_only_ignores_comments_not_code():
    a = 'int f(int x) { // the input\n  return x + 1; /* one more */ }\nconst char* s = "a // b";\n'
    b = 'int f(int x) {\n  return x + 1;   }\nconst char* s = "a // b";'
    assert counters.code_only(a) == counters.code_only(b)
    assert counters.code_only(a) != counters.code_only(a.replace("x + 1", "x + 2"))
    assert '"a // b"' in counters.code_only(a)

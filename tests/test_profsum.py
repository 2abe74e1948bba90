"""Host logic of the rocprofv3 summaries that bench.py reads back."""
import os

from paper_1603_03590_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size","Kernel_Id",'
       '"Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count","Accum_VGPR_Count",'
       '"SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"\n')


def _csv(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as f:
        f.write(HDR)
        for i, (k, c, v) in enumerate(rows):
            f.write(f'{i},{i},"Agent 1",1,1,1,64,1,"{k}",256,0,0,8,0,16,"{c}",{v},0,1\n')


def test_traffic_record_scales_by_the_copy_probe(tmp_path):
    """Counters scaled so that the copy probe reads back its own size:
    FETCH 2x, WRITE 1x here; with the filter, only launches after the last
    persistent-level launch count."""
    copy = 4 * 1024  # KiB of a 4 MiB copy
    f = [("__amd_rocclr_copyBuffer", "FETCH_SIZE", copy / 2)] * 5 + [
        ("k_level<8, 16>(LevelLaunch)", "FETCH_SIZE", 999.0),
        ("k_phase_refine<8, 8, 512, false>(PhaseLaunch)", "FETCH_SIZE", 100.0),
        ("k_phase_refine<8, 8, 512, false>(PhaseLaunch)", "FETCH_SIZE", 300.0)]
    w = [("__amd_rocclr_copyBuffer", "WRITE_SIZE", copy)] * 5 + [
        ("k_level<8, 16>(LevelLaunch)", "WRITE_SIZE", 999.0),
        ("k_phase_refine<8, 8, 512, false>(PhaseLaunch)", "WRITE_SIZE", 10.0),
        ("k_phase_refine<8, 8, 512, false>(PhaseLaunch)", "WRITE_SIZE", 30.0)]
    _csv(str(tmp_path / "f"), f)
    _csv(str(tmp_path / "w"), w)
    line, rec = profsum.traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), "k_phase_refine<", 4, 7, 1,
                                       after=r"k_level<")
    assert rec["launches"] == 2 and rec["tile"] == 7 and rec["mode"] == 1
    assert abs(rec["fetch_bytes_per_launch"] - 2 * 200.0 * 1024) < 1e-6
    assert abs(rec["write_bytes_per_launch"] - 20.0 * 1024) < 1e-6
    p = tmp_path / "s.md"
    p.write_text("# x\n\n" + line + "\n")
    back = profsum.read_traffic(str(p))
    assert back["tile"] == 7 and back["mode"] == 1 and abs(back["bytes_per_launch"] - rec["bytes_per_launch"]) < 1.0
    assert back["source_sha"] == profsum.source_hash()
    # several records: the one measured with the asked tile and launch mode
    _, rec10 = profsum.traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), "k_phase_refine<", 4, 10, 3,
                                      after=r"k_level<")
    line10 = "traffic: " + " ".join(f"{k}={v}" for k, v in rec10.items())
    p.write_text("# x\n\n" + line + "\n" + line10 + "\n")
    assert profsum.read_traffic(str(p), tile=10, mode=3)["tile"] == 10
    assert profsum.read_traffic(str(p), tile=7, mode=1)["tile"] == 7
    assert profsum.read_traffic(str(p), tile=7, mode=3) is None
    table = profsum.util_table(str(tmp_path / "f"))
    assert "`k_phase_refine<8, 8, 512, false>` | 2 | 200 |" in table and "`k_level<8, 16>` | 1 |" in table
    # without the filter the persistent launch counts too
    _, rec_all = profsum.traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), "k_phase_refine<|k_level<", 4, 7, 1)
    assert rec_all["launches"] == 3


def test_committed_traffic_record_parses():
    rec = profsum.read_traffic(os.path.join(ROOT, "profiles", "refine_c2a_1024x436_hbm_traffic.md"))
    assert rec is not None and rec["bytes_per_launch"] > 0 and "source_sha" in rec

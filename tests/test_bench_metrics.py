"""Host-side metric of the grid-refinement study (bench.grouped_errors, the
grouped relative frequency error of Sec. 7.5), checked on hand-made spectra."""

import numpy as np

from bench import grouped_errors


def test_grouped_errors_plain():
    ref = np.arange(1.0, 41.0) ** 2          # frequencies 1..40
    lam = (np.arange(1.0, 41.0) * 1.01) ** 2  # every frequency 1 % high
    e = grouped_errors(lam, ref, 0, 40)
    assert len(e) == 10 and np.allclose(e, 0.01)


def test_grouped_errors_group_means_and_gamma_exclusion():
    # Gamma: 12 zero modes are not passed in; groups 0..2 hold only zero modes
    ref = np.arange(1.0, 29.0) ** 2
    f = np.arange(1.0, 29.0).copy()
    f[0] *= 1.04   # first non-zero band: group 3 (bands 12..15) sees one 4 % error
    f[27] *= 0.98  # last band: group 9 sees one 2 % error
    e = grouped_errors(f ** 2, ref, 12, 40)
    assert e[:3] == [None, None, None]
    assert abs(e[3] - 0.04 / 4) < 1e-15 and abs(e[9] - 0.02 / 4) < 1e-15
    assert all(abs(x) < 1e-15 for x in e[4:9])


def test_grouped_errors_partial_zero_group():
    # 2 zero modes: group 0 averages its 2 non-zero members only
    ref = np.ones(6)
    lam = np.array([1.21, 1.0, 1.0, 1.0, 1.0, 1.0])  # 10 % frequency error on band 2
    e = grouped_errors(lam, ref, 2, 8)
    assert abs(e[0] - 0.05) < 1e-15 and e[1] == 0.0


def test_profile_summaries_from_csv(tmp_path):
    """bench.kernel_stats and bench.counter_stats on small hand-written
    rocprofv3 csv files: per-kernel rows, per-grid means, counter means."""
    from bench import counter_stats, kernel_stats
    kt = tmp_path / "kt" / "host"
    kt.mkdir(parents=True)
    (kt / "x_kernel_stats.csv").write_text(
        "Name,Calls,TotalDurationNs,AverageNs,Percentage\n"
        "\"void (anonymous namespace)::solve_plane_kernel<64, 16, 512>(SolveArgs, int)\",2,3000,1500,75.0\n"
        "copy_kernel(long),1,1000,1000,25.0\n")
    (kt / "x_kernel_trace.csv").write_text(
        "Kernel_Name,Grid_Size_X,Grid_Size_Y,Grid_Size_Z,Workgroup_Size_X,Start_Timestamp,End_Timestamp\n"
        "\"void (anonymous namespace)::solve_plane_kernel<64, 16, 512>(SolveArgs, int)\",1024,1,1,512,0,1000\n"
        "\"void (anonymous namespace)::solve_plane_kernel<64, 16, 512>(SolveArgs, int)\",1024,1,1,512,5000,7000\n"
        "copy_kernel(long),256,1,1,256,9000,10000\n")
    t = kernel_stats(str(tmp_path / "kt"))
    assert "| solve_plane_kernel<64, 16, 512> | 2 | 1.5 | 0.000 | 75.0 |" in t
    assert "| solve_plane_kernel<64, 16, 512> | (1024, 1, 1) | 512 | 2 | 1.5 |" in t
    assert "Total kernel time 0.000 s." in t
    pm = tmp_path / "pm"
    pm.mkdir()
    (pm / "p_counter_collection.csv").write_text(
        "Kernel_Name,Grid_Size,Workgroup_Size,Counter_Name,Counter_Value\n"
        "\"void (anonymous namespace)::plane_kernel<64, 64, -1, 1>(PlaneArgs)\",393216,512,FETCH_SIZE,100\n"
        "\"void (anonymous namespace)::plane_kernel<64, 64, -1, 1>(PlaneArgs)\",393216,512,FETCH_SIZE,300\n"
        "\"void (anonymous namespace)::plane_kernel<64, 64, -1, 1>(PlaneArgs)\",393216,512,SQ_WAVES,6144\n")
    c = counter_stats([str(pm)])
    assert "| kernel | grid | work-group | dispatches | FETCH_SIZE | SQ_WAVES |" in c
    assert "| plane_kernel<64, 64, -1, 1> | 393216 | 512 | 2 | 200 | 6144 |" in c

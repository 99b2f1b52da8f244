/* Prints the size and field offsets of every public struct of include/dsdp.h,
 * one "struct field offset" line each (field "sizeof" for the size), for
 * tests/test_abi_cpu.py to compare with the Python binding's ctypes mirrors. */
#include <stddef.h>
#include <stdio.h>
#include "dsdp.h"

#define S(T) printf(#T " sizeof %zu\n", sizeof(T))
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))

int main(void)
{
    S(dsdp_atom); F(dsdp_atom, x); F(dsdp_atom, xs_type);
    S(dsdp_box); F(dsdp_box, centre); F(dsdp_box, size); F(dsdp_box, spacing);
    S(dsdp_ligand); F(dsdp_ligand, n_atoms); F(dsdp_ligand, atoms); F(dsdp_ligand, n_frags);
    F(dsdp_ligand, frag_start); F(dsdp_ligand, frag_parent); F(dsdp_ligand, axis); F(dsdp_ligand, n_bonds);
    F(dsdp_ligand, bonds);
    S(dsdp_params); F(dsdp_params, temperature); F(dsdp_params, bfgs_iters); F(dsdp_params, waves_per_chain);
    F(dsdp_params, optimizer); F(dsdp_params, bb_step_max); F(dsdp_params, ls_min_decrease); F(dsdp_params, tune);
    S(dsdp_pose); F(dsdp_pose, quat); F(dsdp_pose, tors); F(dsdp_pose, e_total); F(dsdp_pose, score);
    F(dsdp_pose, chain);
    S(dsdp_dock_stats); F(dsdp_dock_stats, pose_evals); F(dsdp_dock_stats, local_opts); F(dsdp_dock_stats, accepted);
    F(dsdp_dock_stats, n_nonfinite); F(dsdp_dock_stats, kernel_ms); F(dsdp_dock_stats, search_ms);
    S(dsdp_tune_entry); F(dsdp_tune_entry, kind); F(dsdp_tune_entry, plan); F(dsdp_tune_entry, waves_per_chain);
    F(dsdp_tune_entry, trial_steps); F(dsdp_tune_entry, trial_ms);
    S(dsdp_sched_info); F(dsdp_sched_info, completed); F(dsdp_sched_info, resident_receptors);
    F(dsdp_sched_info, pool_bytes); F(dsdp_sched_info, ticks);
    return 0;
}

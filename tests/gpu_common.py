"""GPU-side fixtures: device buffers and library calls for the parity tests.

Every call goes through the C ABI (libdsdp.so) via the package's ctypes binding.
The library must be built; if it is missing on a machine with a GPU the tests fail (they do
not skip).
"""
import numpy as np

import paper_2303_09916_amd as D


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    D.lib()   # raises when the library is not built
    return torch


def dev_bytes(torch, n):
    return torch.empty(max(int(n), 256), dtype=torch.uint8, device="cuda")


class GpuGrid:
    """Maps built by dsdp_build_grids on the current device."""

    def __init__(self, rec_xyz, rec_types, box, map_types):
        torch = torch_cuda()
        self.torch = torch
        self.box = box
        self.map_types = list(map_types)
        self.maps = dev_bytes(torch, D.dsdp_grids_bytes(box, len(map_types)))
        self.ws = dev_bytes(torch, D.dsdp_build_grids_workspace_bytes(len(rec_types), box))
        self.handle = D.dsdp_build_grids(rec_xyz, rec_types, box, map_types, self.maps, self.ws)
        torch.cuda.synchronize()
        self.n, self.origin = D.dsdp_grid_dims(box)

    def maps_host(self):
        nx, ny, nz = self.n
        T = len(self.map_types)
        return self.maps[: nx * ny * nz * T * 16].view(self.torch.float32).cpu().numpy().reshape(T, nz, ny, nx, 4)

    def __del__(self):
        try:
            D.dsdp_grids_release(self.handle)
        except Exception:
            pass


def gpu_eval(grid, lig, poses, params=None):
    torch = grid.torch
    n = len(poses)
    L = D.Ligand.from_synth(lig)
    d_p = torch.from_numpy(np.ascontiguousarray(poses, dtype=np.float32)).cuda()
    d_e = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    d_g = torch.zeros((n, L.D), dtype=torch.float32, device="cuda")
    d_x = torch.zeros((n, L.n_atoms, 3), dtype=torch.float32, device="cuda")
    ws = dev_bytes(torch, D.dsdp_dock_workspace_bytes(L, n))
    D.dsdp_eval_poses(grid.handle, L, d_p, n, d_e, d_g, d_x, ws, params)
    torch.cuda.synchronize()
    return d_e.cpu().numpy(), d_g.cpu().numpy(), d_x.cpu().numpy()


def gpu_local_opt(grid, lig, poses, params=None):
    torch = grid.torch
    n = len(poses)
    L = D.Ligand.from_synth(lig)
    d_p = torch.from_numpy(np.ascontiguousarray(poses, dtype=np.float32)).cuda()
    d_o = torch.zeros_like(d_p)
    d_e = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    d_n = torch.zeros((n,), dtype=torch.int32, device="cuda")
    ws = dev_bytes(torch, D.dsdp_dock_workspace_bytes(L, n))
    D.dsdp_local_opt(grid.handle, L, d_p, n, d_o, d_e, d_n, ws, params)
    torch.cuda.synchronize()
    return d_o.cpu().numpy(), d_e.cpu().numpy(), d_n.cpu().numpy()


def gpu_dock(grid, lig, n_chains, n_steps, seed, top_k, params=None, want_chains=True):
    torch = grid.torch
    L = D.Ligand.from_synth(lig)
    ws = dev_bytes(torch, D.dsdp_dock_workspace_bytes(L, n_chains))
    return D.dsdp_dock(grid.handle, L, n_chains, n_steps, seed, top_k, ws, params, want_chains=want_chains)

"""Device buffers and call sequence for one frame (PyTorch = memory + streams only).

DeviceScene uploads a scenes.Scene once, sizes every output and workspace from
host-known upper bounds (no device readbacks), and enqueues
hm_lod_select -> hm_generate_strands -> hm_raster_vis -> hm_resolve_shade on
the current torch stream.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import hm
from .scenes import ResolveParams, Scene, ShadowParams, light_camera


def _u32(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()


def _f32(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


class DeviceScene:
    def __init__(self, sc: Scene, rparams: Optional[hm.RasterParams] = None,
                 resolve: Optional[ResolveParams] = None, cap: Optional[int] = None,
                 mode: Optional[int] = None):
        import torch
        self.sc = sc
        self.S, self.W, self.H = sc.n_scenes, sc.width, sc.height
        self.fr = hm.frame(self.S, self.W, self.H)
        self.mesh_t = dict(layer_pos=_f32(sc.layer_pos), quads=_u32(sc.quads),
                           bundle_key=_u32(sc.bundle_key), bundle_nstrands=_u32(sc.bundle_nstrands),
                           bundle_cmax=_u32(sc.bundle_cmax), bundle_scene=_u32(sc.bundle_scene))
        self.mesh = hm.hair_mesh(self.mesh_t)
        self.cams = _f32(sc.cams)
        self.scene_z = None if sc.scene_z is None else _f32(sc.scene_z)
        self.strand_base = _u32(sc.strand_base)
        self.strand_rgb = None if sc.strand_rgb is None else _f32(sc.strand_rgb)
        self.cap = int(cap or max(sc.n_cp_full, 2))
        B = sc.n_bundles
        dev = "cuda"
        self.table = torch.zeros((B, 4), dtype=torch.int32, device=dev)
        self.scene_off = torch.zeros(self.S + 1, dtype=torch.int32, device=dev)
        self.totals = torch.zeros(2, dtype=torch.int64, device=dev)
        self.pos_w = torch.zeros((self.cap, 4), dtype=torch.float32, device=dev)
        self.rgb = torch.zeros((self.cap, 4), dtype=torch.float32, device=dev)
        self.flags = torch.zeros(self.cap, dtype=torch.uint8, device=dev)
        self.vis = torch.zeros((self.S, 2, self.H, self.W), dtype=torch.int64, device=dev)
        self.out = torch.zeros((self.S, self.H, self.W, 4), dtype=torch.float32, device=dev)
        self.rparams = rparams or hm.raster_defaults(self.fr)
        self.rparams.r_min = sc.r_min
        self.resolve_params = resolve or ResolveParams()
        self.mode = sc.mode if mode is None else mode
        self.sp = hm.shade_params(self.resolve_params, self.mode, sc.bg)
        self.gp = hm.GenParams(sc.seed, sc.strand_width, sc.curl_amp, sc.curl_turns,
                               (ctypes_f3(sc.base_rgb)))
        self.ws_lod = torch.zeros(hm.workspace_size(hm.CALL_LOD, self.fr, n_bundles=B),
                                  dtype=torch.uint8, device=dev)
        self.ws_raster = torch.zeros(
            hm.workspace_size(hm.CALL_RASTER, self.fr, cap=self.cap, rparams=self.rparams),
            dtype=torch.uint8, device=dev)
        self.ws_resolve = torch.zeros(max(hm.workspace_size(hm.CALL_RESOLVE, self.fr), 1),
                                      dtype=torch.uint8, device=dev)
        self.st = hm.strands(self.pos_w, self.rgb, self.flags, self.scene_off, self.cap)

    def set_raster_params(self, rp: hm.RasterParams):
        import torch
        rp.r_min = self.sc.r_min
        need = hm.workspace_size(hm.CALL_RASTER, self.fr, cap=self.cap, rparams=rp)
        if need > self.ws_raster.numel():
            self.ws_raster = torch.zeros(need, dtype=torch.uint8, device="cuda")
        self.rparams = rp

    # ------------------------------------------------------------ steps
    def lod(self):
        hm.lod_select(self.mesh, self.cams, self.fr, self.sc.lod_mode, self.sc.lod_lambda,
                      self.sc.seed, self.table, self.scene_off, self.totals, self.ws_lod)

    def generate(self):
        hm.generate_strands(self.mesh, self.table, self.strand_base, self.strand_rgb, self.gp,
                            self.st)

    def raster(self):
        hm.raster_vis(self.st, self.cams, self.fr, self.rparams, self.scene_z, self.vis,
                      self.ws_raster)

    def generate_raster_tiled(self):
        """Generation that bins as it assembles, then the tiled raster (one
        call; the same stream and vis as generate() + raster())."""
        import torch
        need = hm.workspace_size(hm.CALL_GEN_RASTER, self.fr, n_bundles=self.sc.n_bundles,
                                 cap=self.cap, rparams=self.rparams)
        ws = getattr(self, "ws_gen_raster", None)
        if ws is None or ws.numel() < need:
            self.ws_gen_raster = torch.zeros(need, dtype=torch.uint8, device="cuda")
        hm.generate_raster_tiled(self.mesh, self.table, self.strand_base, self.strand_rgb,
                                 self.gp, self.st, self.cams, self.fr, self.rparams,
                                 self.scene_z, self.vis, self.ws_gen_raster)

    def use_gbuffer(self, on: bool = True):
        """Compressed G-buffer keys (depth | tangent, albedo, AO) instead of
        segment ids; the resolve then shades each centre hit from its key
        alone (centre mode)."""
        rp = hm.RasterParams.from_buffer_copy(self.rparams)
        rp.payload = hm.PAYLOAD_GBUFFER if on else hm.PAYLOAD_SEGMENT
        self.set_raster_params(rp)
        self.sp.payload = rp.payload
        if on:
            self.sp.mode = hm.RESOLVE_CENTER
            self.mode = hm.RESOLVE_CENTER

    def _stream_desc(self, gbuffer: bool) -> hm.Strands:
        """The stream descriptor of a call; with G-buffer keys the calls read
        and write no control point, so its arrays are NULL."""
        if not gbuffer:
            return self.st
        return hm.Strands(None, None, None, self.scene_off.data_ptr(), self.S, self.cap)

    def generate_raster(self):
        """Generation and raster in one pass (fused, direct atomics); with
        G-buffer keys (use_gbuffer) no stream is written."""
        gb = self.rparams.payload == hm.PAYLOAD_GBUFFER
        hm.generate_raster(self.mesh, self.table, self.strand_base, self.strand_rgb, self.gp,
                           self._stream_desc(gb), self.cams, self.fr, self.rparams.r_min,
                           self.scene_z, self.vis, payload=self.rparams.payload)

    def render_fused(self):
        self.lod()
        self.generate_raster()
        self.resolve()
        return self.out

    def resolve(self, out=None):
        hm.resolve_shade(self._stream_desc(self.sp.payload == hm.PAYLOAD_GBUFFER), self.vis,
                         self.cams, self.fr, self.sp, self.out if out is None else out,
                         self.ws_resolve)

    def render(self):
        self.lod()
        self.generate()
        self.raster()
        self.resolve()
        return self.out

    def render_binned(self):
        """The frame with generation and binning in one pass."""
        self.lod()
        self.generate_raster_tiled()
        self.resolve()
        return self.out

    def shadows(self, shp: ShadowParams):
        """Deep-opacity-map shadows of a single-scene frame (Sec. 3.4 with the
        LOD depth correction of Sec. 3.2.3): the stream is rasterized from the
        light camera, the fragment counts per layer accumulated, and the
        transmittance of every pixel's shaded point computed from the current
        visibility buffer; later resolves are shadowed by it.  Call after
        raster()."""
        import torch
        if self.S != 1:
            raise ValueError("deep opacity maps take a single scene")
        dev = "cuda"
        if getattr(self, "_dom", None) is None or self._dom[0] != shp:
            lfr = hm.frame(1, shp.width, shp.height)
            self._dom = (shp, _f32(light_camera(self.sc, shp, self.resolve_params)),
                         torch.empty((1, 2, shp.height, shp.width), dtype=torch.int64, device=dev),
                         hm.DomParams(shp.width, shp.height, shp.n_layers, shp.layer_codes(),
                                      shp.r_min, shp.alpha),
                         torch.empty((shp.n_layers, shp.height, shp.width), dtype=torch.int32,
                                     device=dev),
                         torch.zeros(hm.workspace_size(hm.CALL_DOM, lfr, cap=self.cap),
                                     dtype=torch.uint8, device=dev),
                         torch.ones((self.H, self.W), dtype=torch.float32, device=dev))
        _, light, lvis, dp, counts, dws, shadow = self._dom
        hm.dom_accumulate(self.st, light, dp, lvis, counts, dws)
        hm.dom_shadow(self.st, self.vis, self.cams, self.fr, light, dp, lvis, counts, self.table,
                      self.mesh_t["bundle_nstrands"], shadow)
        self.light_cam, self.light_vis, self.dom_counts, self.shadow = light, lvis, counts, shadow
        self.sp.shadow = hm._ptr(shadow)
        return shadow

    def render_shadowed(self, shp: ShadowParams):
        self.lod()
        self.generate()
        self.raster()
        self.shadows(shp)
        self.resolve()
        return self.out

    # ------------------------------------------------------------ whole frame
    def frame_desc(self) -> hm.FrameDesc:
        d = hm.FrameDesc()
        d.mesh = self.mesh
        d.cams = hm._ptr(self.cams)
        d.frame = self.fr
        d.lod = hm.LodParams(self.sc.lod_mode, self.sc.lod_lambda, self.sc.seed)
        d.table = hm._ptr(self.table)
        d.ws_lod, d.ws_lod_bytes = hm._ptr(self.ws_lod), self.ws_lod.numel()
        d.strand_base = hm._ptr(self.strand_base)
        d.strand_rgb = hm._ptr(self.strand_rgb)
        d.gen = self.gp
        d.strands = self.st
        d.totals = hm._ptr(self.totals)
        d.raster = self.rparams
        d.scene_z = hm._ptr(self.scene_z)
        d.vis = hm._ptr(self.vis)
        d.ws_raster, d.ws_raster_bytes = hm._ptr(self.ws_raster), self.ws_raster.numel()
        d.shade = self.sp
        d.out_rgba = hm._ptr(self.out)
        d.ws_resolve, d.ws_resolve_bytes = hm._ptr(self.ws_resolve), self.ws_resolve.numel()
        return d

    def render_native(self):
        """The whole frame through one C call (hm_render_frame)."""
        hm.render_frame(self.frame_desc())
        return self.out

    def capture_graph(self) -> hm.Graph:
        """Capture the frame into a HIP graph on the current (non-default) stream."""
        import torch
        h = torch.cuda.current_stream().cuda_stream
        if not h:
            raise RuntimeError("capture needs a non-default stream (use torch.cuda.stream)")
        return hm.Graph(self.frame_desc(), h)

    # ------------------------------------------------------------ host views
    def n_cp(self) -> int:
        return int(self.totals[1].item())

    def host_stream(self):
        n = min(self.n_cp(), self.cap)
        return (self.pos_w[:n].cpu().numpy(), self.rgb[:n].cpu().numpy(),
                self.flags[:n].cpu().numpy())

    def host_vis(self) -> np.ndarray:
        return self.vis.cpu().numpy().view(np.uint64)


def ctypes_f3(v):
    import ctypes
    return (ctypes.c_float * 3)(*[float(x) for x in v])
